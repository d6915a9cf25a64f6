// sfq.hip -- HIP kernels and the C ABI (include/sfq.h) of the MI355X QED Monte Carlo step.
//
// Method: Montefiori & Tamburini, arXiv:2301.07684 (SFQEDtoolkit); see sfq_device.h for the
// equation behind every device function.
//
// Kernel design (gfx950, wave64):
//   bulk_kernel  persistent streaming pass over all tiles of a step: coalesced FP64 SoA loads
//                in one group per iteration, the fields (arrays, one uniform value, or a plane
//                wave computed here), the optional Boris push, gamma, chi, the rate from
//                LDS-staged coefficient tables and the decision (or the beyond-LCFA force
//                update); emitters are compacted with a wave ballot + popcount prefix into the
//                block's own slice of a queue (one LDS atomic per wave, no global atomics).  It
//                writes every slot of a chunk it updates (whole cache lines), addresses each
//                chunk from its first element (scalar bases, one 32-bit lane offset), and
//                carries none of the sampling code, so its register footprint stays small.
//   emit_kernel  each queue slice is sampled by a few blocks with all lanes busy: Philox draws,
//                the inverse-CDF tables (L2-resident), recoil and products.  Each block's
//                product slots come from the queued counts of every earlier slice, which it
//                sums itself; block 0 adds the step's counters once and the last block out
//                advances the product counts (per-wave reservations only for beyond-LCFA
//                photons and per-set products).
//   defer_kernel the shares the streaming pass deferred (queue too small), stepped whole.
//   rates/chi/sample/philox kernels: grid-stride elementwise kernels behind the batched calls.
#include <hip/hip_runtime.h>

#include <dlfcn.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/sfq.h"
#include "sfq_device.h"

using namespace sfq;

// =============================================================================================
// Kernel arguments
// =============================================================================================
struct Tables {
    const double *rad, *pair, *ka, *kb, *phinv, *ppinv;
    const float *rad32, *pair32, *phinv32, *ppinv32;
    int trunc;           // evaluate the truncated form of the inverse patches (sfq_config.approx)
};

struct Physics {
    double dt;
    double lc_over_lr;   // lambda_C/lambda_r: chi = gamma lc |...|, tau_C in units of 1/omega_r
    double k_rate;       // alpha/(sqrt3 pi) lambda_r/lambda_C
    double chi_min_pair; // 0.01, or 0.3 with bw_fast
    int trunc;           // evaluate the truncated form of the rate segments (sfq_config.approx)
};

struct StepArgs {
    Tables tb;
    Physics ph;
    const sfq_tile* tiles;
    const uint32_t* chunk_off;  // [ntiles + 1], prefix sums of chunks per tile
    int ntiles;
    int nchunks;
    int chunk;
    int decision;
    int blcfa;
    uint32_t step;
    const unsigned long long* step_ptr;  // if set, the step index is read from device memory
    uint64_t seed;
    // emitter queue (SoA).  Wave w of streaming block b owns the slice s = STEP_WAVES b + w,
    // entries [s cap, (s+1) cap): leptons from the start of the slice upwards, photons from its
    // end downwards.
    uint32_t* q_idx;
    uint32_t* q_tile;
    double* q_chi;
    double* q_gamma;
    double* q_px;
    double* q_py;
    double* q_pz;
    uint64_t* q_uid;
    double* q_aux;              // beyond-LCFA tau/tau_C for the threshold (negative: LCFA)
    double* q_aux2;             // beyond-LCFA: gamma of the pushed momentum minus gamma^{(n)}
    uint32_t* q_count;          // [2 slices]: lepton and photon emitters queued in each slice
    uint32_t* q_sbcount;        // [4 grid]: per streaming block its slices' two sums, the chunks
                                // it took and a spare word
    unsigned long long* q_proc; // [grid]: particles processed by each block of the streaming pass
    uint64_t q_cap_per_wave;    // entries of one slice
    // Shares that did not fit: a wave whose slice could not take every particle of its share of
    // a chunk (STEP_BLOCK/64 waves share a chunk) leaves that share untouched and appends
    // chunk * STEP_WAVES + wave here; the emitter kernel steps those shares afterwards.
    uint32_t* d_list;
    unsigned* d_ctl;            // [5]: shares deferred, next share to step, deferred-share
                                // blocks done, emitter blocks done, next chunk to stream
    unsigned* obs;              // nullable, host-mapped: [0] the largest emitter fraction of a
                                // wave's share (float bits), [1] shares deferred (for sizing)
    unsigned* emit_obs;         // nullable, host-mapped: the step's emitters over the particles
                                // it processed (float bits; picks the emitter pass's grid)
    int grid;                   // blocks of the streaming kernel (STEP_WAVES slices each)
    int max_chunks;             // the most chunks one streaming block takes (the queue's worst
                                // case is sized for it)
    int emit_split;             // emitter blocks per streaming block's slices
    int may_defer;              // the slices are smaller than the step's worst case (host side:
                                // the deferred-share kernel is enqueued)
    sfq_products prod[3];       // photons, electrons, positrons
    unsigned long long* prod_counts;
    sfq_counters* counters;
    const sfq_product_set* sets; // nsets > 0: per-tile product destinations (device copy)
    int nsets;
    int push;                    // leptons get the Boris push before the step
    int wave;                    // some tile gives its fields as a plane wave
    int zero_counts;             // the step's product counts start from zero (nsets == 0: the
                                 // emitter kernel takes the bases as 0 instead of reading them)
};

enum { CNT_PROCESSED, CNT_EMITTED, CNT_CONVERTED, CNT_REJECTED, CNT_OOD, CNT_CLAMPED, CNT_OVERFLOW,
       CNT_DEFERRED, CNT_N };

// =============================================================================================
// Device helpers shared by the step and the batched calls
// =============================================================================================
template <bool MIXED>
__device__ __forceinline__ double rate_lepton(const void* rad, const Physics& ph, double gamma,
                                              double chi, bool* ood)
{
    if (!(chi > 0.0) || !(gamma > 0.0)) return 0.0;
    if (MIXED) {
        const float wt = wtilde_rad((const float*)rad, (float)chi, ood, ph.trunc != 0);
        return (double)((float)ph.k_rate * (float)chi / (float)gamma * wt);
    }
    const double wt = wtilde_rad((const double*)rad, chi, ood, ph.trunc != 0);
    return ph.k_rate * chi * rcp_nr(gamma) * wt;
}

template <bool MIXED>
__device__ __forceinline__ double rate_photon(const void* pair, const Physics& ph, double gamma,
                                              double chi, bool* ood)
{
    if (!(chi >= ph.chi_min_pair) || !(gamma > 0.0)) return 0.0;
    if (MIXED) {
        const float wt = wtilde_pair((const float*)pair, (float)chi, ood, ph.trunc != 0);
        return (double)((float)ph.k_rate / (float)gamma * wt);
    }
    const double wt = wtilde_pair((const double*)pair, chi, ood, ph.trunc != 0);
    return ph.k_rate * rcp_nr(gamma) * wt;
}

// Energy sampling for one lane; every lane of the wave must call it (cooperative table
// evaluation).  Lanes with valid == false pass through with a dummy request.
//   photon emission (pair == false): s = 3 chi wbar^3 / 2 (Eq. (subs_altri)); the photon takes
//     the energy fraction s/(1+s), the emitter keeps 1/(1+s)
//   pair creation (pair == true): v = vbar of Eq. (again_pp) and 1 - v without cancellation
// MIXED evaluates in FP32 and re-evaluates in FP64 the lanes whose energy fraction exceeds
// 0.999 (photon: s > 999; pair: (1 + v)/2 > 0.999).
template <bool MIXED>
__device__ __forceinline__ void sample_coop(const Tables& tb, bool valid, bool pair, double chi,
                                            double r, double& s_out, double& v_out,
                                            double& omv_out, bool& ood)
{
    const double u = pair ? fabs(2.0 * r - 1.0) : r;   // 2r - 1 is exact
    InvReq q;
    if (!valid) q = photon_req(1.0, 0.25);
    else if (pair) q = pair_req(chi, u);
    else q = photon_req(chi, u);
    ood = valid && q.ood;
    const int patch = q.patch + (pair ? N_INV_CHI * N_R_SEG : 0);  // pair patches follow
    bool need64 = true;
    if (MIXED) {
        const float f = coop_patch_eval<float>(tb.phinv32, patch, (float)q.Xr, (float)q.Xc, valid,
                                               tb.trunc != 0);
        const float uf = (float)u;
        if (!pair) {
            const float xbar = q.upper ? expf(f) : (f * uf) * (f * uf) * (f * uf);
            const float s = 1.5f * (float)chi * xbar;
            s_out = (double)s;
            need64 = !(s <= 999.0f);
        } else {
            const float y = q.upper ? expf(f) : (f * uf) * (f * uf);
            const float eta0 = (float)(8.0 / (3.0 * chi));
            const float den = y + eta0;
            const float v = sqrtf(y / den);
            v_out = (double)v;
            omv_out = (double)((eta0 / den) / (1.0f + v));
            need64 = !(v <= 0.998f);
        }
        need64 = need64 && valid;
        if (__ballot(need64) == 0) return;
    }
    need64 = need64 && valid;
    const double f = coop_patch_eval<double>(tb.phinv, patch, q.Xr, q.Xc, need64, tb.trunc != 0);
    if (!need64) return;
    if (!pair) {
        const double w = f * u;
        const double xbar = q.upper ? exp(f) : w * w * w;
        s_out = 1.5 * chi * xbar;
    } else {
        const double w = f * u;
        const double y = q.upper ? exp(f) : w * w;
        const double eta0 = 8.0 / (3.0 * chi);
        const double den = y + eta0;
        const double v = sqrt(y / den);
        v_out = v;
        omv_out = (eta0 / den) / (1.0 + v);
    }
}

// electron and positron energies from v (Eq. (return_to_nrg)): the electron takes (1 + v)/2
// of the photon energy when r' = 2r - 1 >= 0, (1 - v)/2 otherwise
__device__ __forceinline__ void pair_energies(double gamma, double r, double v, double omv,
                                              double& ge, double& gp)
{
    const double hi = 0.5 * gamma * (1.0 + v), lo = 0.5 * gamma * omv;
    if (2.0 * r - 1.0 < 0.0) { ge = lo; gp = hi; } else { ge = hi; gp = lo; }
}

__device__ __forceinline__ double lepton_momentum_factor(double g, double pn, bool& clamped)
{
    if (g > 1.0 && pn > 0.0) {
        clamped = false;
        return sqrt((g - 1.0) * (g + 1.0)) / pn;
    }
    clamped = true;
    return 0.0;
}

__device__ __forceinline__ int lane_id() { return __lane_id(); }

// streaming accesses of the particle arrays: read once per step, so they are marked
// non-temporal and do not push the emitter queue out of the caches
#ifndef SFQ_NT
#define SFQ_NT 1
#endif
// (the pointers come from descriptors in memory, so they are cast to the global address space
// to get global rather than flat memory instructions)
template <typename T>
__device__ __forceinline__ T ld_stream(const T* p)
{
    const __attribute__((address_space(1))) T* g = (const __attribute__((address_space(1))) T*)p;
#if SFQ_NT
    return __builtin_nontemporal_load(g);
#else
    return *g;
#endif
}
template <typename T>
__device__ __forceinline__ void st_stream(T* p, T v)
{
    __attribute__((address_space(1))) T* g = (__attribute__((address_space(1))) T*)p;
#if SFQ_NT
    __builtin_nontemporal_store(v, g);
#else
    *g = v;
#endif
}

// A streaming load or store at a uniform base plus a 32-bit lane byte offset: the particle
// loops address a chunk (at most 2^22 particles) from its first element, so that every array
// access is a global instruction with a scalar base and one shared 32-bit offset register,
// with no 64-bit address arithmetic per array and lane.
template <typename T>
__device__ __forceinline__ T ld_off(const T* base, uint32_t byte_off)
{
    return ld_stream((const T*)((const char*)base + byte_off));
}
template <typename T>
__device__ __forceinline__ void st_off(T* base, uint32_t byte_off, T v)
{
    st_stream((T*)((char*)base + byte_off), v);
}

// wave-aggregated reservation of `want` slots on a global counter; returns this lane's slot
__device__ __forceinline__ unsigned long long wave_reserve(unsigned long long* counter, bool want)
{
    const unsigned long long mask = __ballot(want);
    if (mask == 0) return 0;
    const int leader = __ffsll((long long)mask) - 1;
    const int lane = lane_id();
    unsigned long long base = 0;
    if (lane == leader) base = atomicAdd(counter, (unsigned long long)__popcll(mask));
    base = __shfl(base, leader);
    const unsigned long long below = mask & ((1ull << lane) - 1ull);
    return base + (unsigned long long)__popcll(below);
}

// Slots in per-owner product buffers: the lanes of a wave that want a slot are grouped by their
// set index (usually one or two distinct sets per wave) and each group takes its slots with one
// atomic.  Every lane of the wave must call this (the loop is wave-uniform).
__device__ __forceinline__ unsigned long long keyed_reserve(const sfq_product_set* sets,
                                                            int species, int key, bool want)
{
    unsigned long long pending = __ballot(want);
    const int lane = lane_id();
    unsigned long long slot = 0;
    while (pending) {
        const int leader = __ffsll((long long)pending) - 1;
        const int lk = __shfl(key, leader);
        const unsigned long long m = __ballot(want && key == lk);
        unsigned long long base = 0;
        if (lane == leader)
            base = atomicAdd(&sets[lk].product_counts[species], (unsigned long long)__popcll(m));
        base = __shfl(base, leader);
        if ((m >> lane) & 1ull) slot = base + (unsigned long long)__popcll(m & ((1ull << lane) - 1ull));
        pending &= ~m;
    }
    return slot;
}

// =============================================================================================
// The step: a streaming kernel over all tiles and an emitter kernel over its compacted queue
// =============================================================================================
constexpr int STEP_BLOCK = 256;
// minimum waves per SIMD requested from the register allocator for the two step kernels.  The
// streaming kernel's register budget decides how many waves can hide HBM latency: the LCFA
// array forms, with their two-particles-per-lane loop, fit 4 waves (FP64) and 5 (mixed); the
// launch shapes that run best use 2 per SIMD (2 blocks of 4 waves per compute unit), with two
// independent particles per lane.  The beyond-LCFA forms
// (which leave the emission threshold's transcendentals to the emitter pass) fit 5 waves
// (mixed), 4 (mixed with the push, FP64) or 3 (FP64 with the push).  The kernels that take
// plane-wave tiles (fields computed in the kernel, two particles per lane in the LCFA loop)
// get 4 waves (LCFA) or 3 (beyond-LCFA).
#ifdef SFQ_BULK_WAVES
constexpr int bulk_waves(bool, bool, bool, bool) { return SFQ_BULK_WAVES; }
#else
constexpr int bulk_waves(bool mixed, bool blcfa, bool push, bool wave)
{
    if (blcfa) return wave ? 3 : (mixed ? (push ? 4 : 5) : (push ? 3 : 4));
    return wave ? 4 : (mixed ? 5 : 4);
}
#endif
#ifndef SFQ_EMIT_WAVES
#define SFQ_EMIT_WAVES 3
#endif
// Emitters dense: above this fraction of a streaming block's particles the emitter kernel
// writes the block's products with non-temporal stores, and above it for the whole step the
// next step's emitter pass runs twice the blocks per compute unit (both measured faster at
// 10-13 % emitters and slower at 2 %).
constexpr float DENSE_EMITTER_FRACTION = 0.06f;

// read as the alive flag of tiles that have no alive array
__device__ const uint8_t k_alive_one[1] = {1};

// A value that is the same in every lane, moved to scalar registers (the tile descriptor is
// fetched with vector loads; keeping its pointers in vector registers would cost two per lane
// each).
__device__ __forceinline__ uint64_t uniform64(uint64_t v)
{
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return ((uint64_t)hi << 32) | lo;
}

template <typename P>
__device__ __forceinline__ P* uniform_ptr(P* p)
{
    return (P*)uniform64((uint64_t)p);
}

__device__ __forceinline__ double uniform_f64(double v)
{
    return __longlong_as_double((long long)uniform64((uint64_t)__double_as_longlong(v)));
}

__device__ __forceinline__ sfq_tile uniform_tile(const sfq_tile& src)
{
    sfq_tile T;
    T.species = (int32_t)__builtin_amdgcn_readfirstlane((uint32_t)src.species);
    T.product_set = (int32_t)__builtin_amdgcn_readfirstlane((uint32_t)src.product_set);
    T.n = uniform64(src.n);
    T.px = uniform_ptr(src.px); T.py = uniform_ptr(src.py); T.pz = uniform_ptr(src.pz);
    T.ex = uniform_ptr(src.ex); T.ey = uniform_ptr(src.ey); T.ez = uniform_ptr(src.ez);
    T.bx = uniform_ptr(src.bx); T.by = uniform_ptr(src.by); T.bz = uniform_ptr(src.bz);
    T.tau = uniform_ptr(src.tau);
    T.uid = uniform_ptr(src.uid);
    T.alive = uniform_ptr(src.alive);
    T.px_prev = uniform_ptr(src.px_prev); T.py_prev = uniform_ptr(src.py_prev);
    T.pz_prev = uniform_ptr(src.pz_prev);
    T.fperp = uniform_ptr(src.fperp);
    T.dfperp = uniform_ptr(src.dfperp);
    T.just_created = uniform_ptr(src.just_created);
    T.chi_out = uniform_ptr(src.chi_out);
    T.rate_out = uniform_ptr(src.rate_out);
    T.step_offset = uniform64(src.step_offset);
    T.field_mode = (int32_t)__builtin_amdgcn_readfirstlane((uint32_t)src.field_mode);
    return T;
}

// A tile's plane wave (field_mode SFQ_FIELDS_PLANE_WAVE), in scalar registers.
struct Wave {
    const double *amp, *phase;
    double k[3], pol[3], phase0;
};

__device__ __forceinline__ Wave uniform_wave(const sfq_tile& src)
{
    Wave w;
    w.amp = uniform_ptr(src.wave_amp);
    w.phase = uniform_ptr(src.wave_phase);
    for (int k = 0; k < 3; ++k) {
        w.k[k] = uniform_f64(src.wave_k[k]);
        w.pol[k] = uniform_f64(src.wave_pol[k]);
    }
    w.phase0 = uniform_f64(src.wave_phase0);
    return w;
}

// Fields of a linearly polarised plane wave at a particle of amplitude a and phase ph:
// E = a cos(ph + theta) e, B = k x E (units m c omega_r / e, so |B| = |E|); phases below
// 2^20 pi/2 in magnitude (the domain of cos_cw).
__device__ __forceinline__ void plane_wave_fields(const Wave& w, double a, double ph, double& ex,
                                                  double& ey, double& ez, double& bx, double& by,
                                                  double& bz)
{
    const double c = a * cos_cw(ph + w.phase0);
    ex = c * w.pol[0];
    ey = c * w.pol[1];
    ez = c * w.pol[2];
    bx = w.k[1] * ez - w.k[2] * ey;
    by = w.k[2] * ex - w.k[0] * ez;
    bz = w.k[0] * ey - w.k[1] * ex;
}

__device__ __forceinline__ int find_tile(const uint32_t* off, int ntiles, int c)
{
    int lo = 0, hi = ntiles - 1;
    while (lo < hi) {  // last t with off[t] <= c (tiles without chunks are skipped)
        const int mid = (lo + hi + 1) >> 1;
        if ((int)off[mid] <= c) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Sum over the block (every thread gets it); s_tmp: at least one word of shared memory, which
// the caller must not be using.
__device__ __forceinline__ unsigned long long block_sum(unsigned long long* s_tmp,
                                                        unsigned long long v)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o);
    __syncthreads();
    if (threadIdx.x == 0) s_tmp[0] = 0;
    __syncthreads();
    if (lane_id() == 0 && v) atomicAdd(&s_tmp[0], v);
    __syncthreads();
    const unsigned long long r = s_tmp[0];
    __syncthreads();
    return r;
}

// Sums of two values over the block (every thread gets both); s_tmp: two words of shared
// memory the caller is not using.
__device__ __forceinline__ void block_sum2(unsigned long long* s_tmp, unsigned long long& a,
                                          unsigned long long& b)
{
    for (int o = 32; o > 0; o >>= 1) {
        a += __shfl_down(a, o);
        b += __shfl_down(b, o);
    }
    __syncthreads();
    if (threadIdx.x == 0) s_tmp[0] = s_tmp[1] = 0;
    __syncthreads();
    if (lane_id() == 0) {
        if (a) atomicAdd(&s_tmp[0], a);
        if (b) atomicAdd(&s_tmp[1], b);
    }
    __syncthreads();
    a = s_tmp[0];
    b = s_tmp[1];
    __syncthreads();
}

__device__ __forceinline__ void block_add_counters(unsigned long long* s_cnt,
                                                   sfq_counters* global,
                                                   const unsigned long long (&vals)[CNT_N])
{
#pragma unroll
    for (int k = 0; k < CNT_N; ++k) {
        unsigned long long v = vals[k];
        for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o);
        if (lane_id() == 0 && v) atomicAdd(&s_cnt[k], v);
    }
    __syncthreads();
    if (threadIdx.x < CNT_N && s_cnt[threadIdx.x])
        atomicAdd(&global->processed + threadIdx.x, s_cnt[threadIdx.x]);
}

// =============================================================================================
// Emitter work of one lane (wave-cooperative: every lane of the wave calls it; lanes with
// valid == false pass through): Philox draws, the energy sample, recoil written in place and
// the products.  Product slots come from the caller (k_ph, k_el, k_po: this lane's slots), or,
// with atomic_slots (and always for beyond-LCFA photons and per-set products), from one atomic
// per wave and buffer; nt_prod (uniform over the wave) writes the products non-temporally.
// =============================================================================================
struct EmitCounts {
    unsigned long long emit = 0, conv = 0, rej = 0, clamp = 0, over = 0, ood = 0;
};

// One product into slot k of a product buffer; nt: non-temporal stores (the emitter kernel uses
// them where emitters are dense, see emit_item)
__device__ __forceinline__ void store_product(const sfq_products& P, unsigned long long k,
                                              double px, double py, double pz, double tau,
                                              uint64_t uid, uint64_t parent, bool nt)
{
    if (nt) {
        st_stream(&P.px[k], px); st_stream(&P.py[k], py); st_stream(&P.pz[k], pz);
        st_stream(&P.tau[k], tau); st_stream(&P.uid[k], uid); st_stream(&P.parent[k], parent);
    } else {
        P.px[k] = px; P.py[k] = py; P.pz[k] = pz;
        P.tau[k] = tau; P.uid[k] = uid; P.parent[k] = parent;
    }
}

template <bool MIXED, bool BLCFA, bool LOCAL>
__device__ __forceinline__ void emit_one(const StepArgs& A, bool valid, bool pair, uint32_t i,
                                         int t, double chi, double gamma, double px, double py,
                                         double pz, uint64_t quid, double tau_ratio,
                                         double dgamma_push, uint32_t base_step,
                                         bool atomic_slots, unsigned long long k_ph,
                                         unsigned long long k_el, unsigned long long k_po,
                                         EmitCounts& C, bool nt_prod)
{
    static_assert(LOCAL || !BLCFA, "beyond-LCFA steps use local decisions");
    const bool multi = A.nsets > 0;
    bool want_ph = false, want_pair = false;
    double pgx = 0, pgy = 0, pgz = 0, tau_a = 0, pbx = 0, pby = 0, pbz = 0, tau_b = 0;
    uint64_t uid_a = 0, uid_b = 0, parent = 0;
    pair = valid && pair;
    uint64_t uid = 0;
    uint32_t step = base_step;
    int pset = 0;
    double r = 0.5;
    if (!valid) { chi = 1.0; gamma = 1.0; px = py = pz = 0.0; }
    Draw d1{0, 0}, d2{0, 0};
    if (valid) {
        // with optical-depth decisions the streaming pass did not read the id (a non-temporal
        // load: the scattered line is not kept in the caches)
        uid = LOCAL ? quid : ld_stream(&A.tiles[t].uid[i]);
        step = base_step + (uint32_t)A.tiles[t].step_offset;
        d1 = philox_draw(A.seed, uid, step, SFQ_P_EMIT);
        d2 = philox_draw(A.seed, uid, step, SFQ_P_CHILD);
        r = uniform53(d1.a);
    }
    double s = 0.0, v = 0.0, omv = 1.0;
    bool ood = false;
    sample_coop<MIXED>(A.tb, valid, pair, chi, r, s, v, omv, ood);
    if (valid) {
        const sfq_tile& T = A.tiles[t];
        if (multi) pset = T.product_set;
        parent = uid;
        const double pn = sqrt(fma(px, px, fma(py, py, pz * pz)));
        if (!pair) {
            const double gph = gamma * (s / (1.0 + s));
            bool accept = true, none = false;
            double gem = gamma / (1.0 + s);
            if (BLCFA) {
                // the threshold gamma_{gamma,LCFA} (Eq. gammaLCFA) from the queued tau/tau_C
                double limit = 0.0;
                if (tau_ratio >= 0.0) {
                    const double arg = chi / (8.0 * gamma) * tau_ratio;
                    limit = 0.7 * gamma /
                            (1.0 + 4.0 / (3.0 * PI * chi) * sinh(3.0 * asinh(arg)));
                }
                // no emission at all when the threshold reaches 0.75 gamma (Sec. 5; it
                // cannot for finite input, as the threshold is at most 0.7 gamma)
                none = !(limit < 0.75 * gamma);
                if (none) {
                    accept = false;
                } else if (!(gph > limit)) {  // Eq. (rej_cond)
                    const Draw dl = philox_draw(A.seed, uid, step, SFQ_P_LOCAL);
                    const double r2 = uniform53(dl.b);
                    const double lp_s = log_photon_pdf(A.tb.ka, A.tb.kb, gph, gamma, chi);
                    const double lp_l = log_photon_pdf(A.tb.ka, A.tb.kb, limit, gamma, chi);
                    accept = log(r2) + lp_s <= lp_l;
                }
                // the pushed momentum recoils by the photon energy
                gem += dgamma_push;
            }
            if (accept) {
                bool cl;
                const double f = lepton_momentum_factor(gem, pn, cl);
                C.clamp += cl ? 1 : 0;
                T.px[i] = px * f; T.py[i] = py * f; T.pz[i] = pz * f;
                if (A.decision == SFQ_OPTICAL_DEPTH) T.tau[i] = optical_depth(d1.b);
                const double fg = pn > 0.0 ? gph / pn : 0.0;
                pgx = px * fg; pgy = py * fg; pgz = pz * fg;
                tau_a = optical_depth(d2.a);
                uid_a = d2.b;
                want_ph = true;
                ++C.emit;
            } else {
                // rejected: the lepton keeps the pushed momentum, which the streaming pass
                // has already written to the tile with the fused push
                if (!none) ++C.rej;
            }
        } else {
            const Draw d3 = philox_draw(A.seed, uid, step, SFQ_P_CHILD2);
            double ge, gp;
            pair_energies(gamma, r, v, omv, ge, gp);
            bool c1, c2;
            const double fe = lepton_momentum_factor(ge, pn, c1);
            const double fp = lepton_momentum_factor(gp, pn, c2);
            C.clamp += (c1 ? 1 : 0) + (c2 ? 1 : 0);
            pgx = px * fe; pgy = py * fe; pgz = pz * fe;   // electron
            pbx = px * fp; pby = py * fp; pbz = pz * fp;   // positron
            tau_a = optical_depth(d1.b);
            uid_a = d2.b;
            tau_b = optical_depth(d2.a);
            uid_b = d3.a;
            if (T.alive) T.alive[i] = 0;
            want_pair = true;
            ++C.conv;
        }
        C.ood += ood ? 1 : 0;
    }
    {
        unsigned long long k;
        if (multi) k = keyed_reserve(A.sets, 0, pset, want_ph);
        else k = (BLCFA || atomic_slots) ? wave_reserve(&A.prod_counts[0], want_ph) : k_ph;
        if (want_ph) {
            const sfq_products P = multi ? A.sets[pset].photons : A.prod[0];
            if (k < P.capacity) {
                store_product(P, k, pgx, pgy, pgz, tau_a, uid_a, parent, nt_prod);
            } else {
                ++C.over;
            }
        }
    }
    unsigned long long ke = k_el, kp = k_po;
    if (multi) {
        ke = keyed_reserve(A.sets, 1, pset, want_pair);
        kp = keyed_reserve(A.sets, 2, pset, want_pair);
    } else if (atomic_slots) {
        ke = wave_reserve(&A.prod_counts[1], want_pair);
        kp = wave_reserve(&A.prod_counts[2], want_pair);
    }
    if (want_pair) {
        const sfq_products E = multi ? A.sets[pset].electrons : A.prod[1];
        if (ke < E.capacity) {
            store_product(E, ke, pgx, pgy, pgz, tau_a, uid_a, parent, nt_prod);
        } else {
            ++C.over;
        }
        const sfq_products P = multi ? A.sets[pset].positrons : A.prod[2];
        if (kp < P.capacity) {
            store_product(P, kp, pbx, pby, pbz, tau_b, uid_b, parent, nt_prod);
        } else {
            ++C.over;
        }
    }
}

// =============================================================================================
// Where the streaming pass puts the emitters it finds
// =============================================================================================
// One lane's emitter: what the emitter work needs (the uid only with local decisions, the two
// beyond-LCFA values only for beyond-LCFA leptons).
struct EmitRec {
    uint32_t i;
    double chi, gamma, px, py, pz;
    uint64_t uid;
    double aux, aux2;
};

__device__ __forceinline__ unsigned long long lanes_below() { return (1ull << lane_id()) - 1ull; }

// The streaming kernel's sink: the wave's own slice of the emitter queue, its counts in scalar
// registers (wave-uniform; no atomics).  The caller makes sure, before each chunk, that the
// slice can take every particle of the wave's share of it.
struct QueueSink {
    uint64_t base;   // first entry of the wave's slice
    uint32_t nl, np; // leptons and photons queued so far

    __device__ __forceinline__ void write(const StepArgs& A, uint64_t slot, int t,
                                          const EmitRec& e, bool local, bool aux) const
    {
        A.q_idx[slot] = e.i;
        A.q_tile[slot] = (uint32_t)t;
        A.q_chi[slot] = e.chi;
        A.q_gamma[slot] = e.gamma;
        A.q_px[slot] = e.px;
        A.q_py[slot] = e.py;
        A.q_pz[slot] = e.pz;
        if (local) A.q_uid[slot] = e.uid;
        if (aux) {
            A.q_aux[slot] = e.aux;
            A.q_aux2[slot] = e.aux2;
        }
    }

    template <bool LOCAL>
    __device__ __forceinline__ void put(const StepArgs& A, bool emit, bool photon, bool aux,
                                        int t, const EmitRec& e)
    {
        const unsigned long long mask = __ballot(emit);
        if (!mask) return;
        const unsigned first = photon ? np : nl;
        if (emit) {
            const unsigned rank = first + (unsigned)__popcll(mask & lanes_below());
            const uint64_t slot = photon ? base + A.q_cap_per_wave - 1 - rank : base + rank;
            write(A, slot, t, e, LOCAL, aux);
        }
        if (photon) np += (unsigned)__popcll(mask); else nl += (unsigned)__popcll(mask);
    }

    // two particles per lane (lane l holds particles 2l, 2l + 1), queued in index order
    __device__ __forceinline__ void put2(const StepArgs& A, const bool (&em)[2], bool photon,
                                         int t, const EmitRec (&e)[2])
    {
        const unsigned long long m0 = __ballot(em[0]), m1 = __ballot(em[1]);
        if (!(m0 | m1)) return;
        const unsigned long long below = lanes_below();
        const unsigned r0 = (photon ? np : nl) +
                            (unsigned)(__popcll(m0 & below) + __popcll(m1 & below));
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            if (em[u]) {
                const unsigned rank = r0 + (u == 1 && em[0] ? 1u : 0u);
                const uint64_t slot = photon ? base + A.q_cap_per_wave - 1 - rank : base + rank;
                write(A, slot, t, e[u], false, false);
            }
        }
        const unsigned total = (unsigned)(__popcll(m0) + __popcll(m1));
        if (photon) np += total; else nl += total;
    }
};

// The sink of the deferred shares (stepped inside the emitter kernel): each emitter's work is
// done at once by the wave, with product slots taken by atomics.
template <bool MIXED, bool BLCFA, bool LOCAL>
struct InlineSink {
    EmitCounts* cnt;
    uint32_t base_step;

    template <bool LOCAL_>
    __device__ __forceinline__ void put(const StepArgs& A, bool emit, bool photon, bool aux,
                                        int t, const EmitRec& e)
    {
        (void)aux;
        if (__ballot(emit) == 0) return;
        emit_one<MIXED, BLCFA, LOCAL>(A, emit, photon, e.i, t, e.chi, e.gamma, e.px, e.py, e.pz,
                                      e.uid, e.aux, e.aux2, base_step, true, 0, 0, 0, *cnt,
                                      false);
    }

    __device__ __forceinline__ void put2(const StepArgs& A, const bool (&em)[2], bool photon,
                                         int t, const EmitRec (&e)[2])
    {
#pragma unroll 1
        for (int u = 0; u < 2; ++u) {
            const bool m = u ? em[1] : em[0];
            const EmitRec& r = u ? e[1] : e[0];
            put<false>(A, m, photon, false, t, r);
        }
    }
};

// =============================================================================================
// The streaming pass: per alive particle gamma, chi (or the beyond-LCFA force update), the rate
// from LDS-staged tables and the decision; emitters go to a sink (the wave's queue slice, or,
// for deferred shares, the emitter work itself) through a wave ballot and popcount prefix.
//
// Memory pattern: each iteration issues all loads of a particle as one group (the alive flag
// included), so an iteration costs one memory round trip.  With optical-depth decisions the
// particle id is not read here: only emitters need it, and the emitter pass fetches it.
//
// Each wave works on its own share of a chunk: lanes are addressed by `tid` (the thread index
// of a 256-thread block: wave w takes tid = 64 w .. 64 w + 63), so any wave can step any
// wave's share of any chunk with the same arithmetic.
// =============================================================================================
constexpr int STEP_WAVES = STEP_BLOCK / 64;

// The LCFA particle loop of a plane-wave chunk, two particles per lane per iteration (see
// stream_chunk for the one-particle loop and its comments; the arithmetic is the same).
template <bool MIXED, bool LOCAL, bool PUSH, typename SINK, typename RT>
__device__ __forceinline__ void lcfa_wave_pairs(const StepArgs& A, const sfq_tile& T,
                                                const Wave& WV, int t, uint64_t start,
                                                uint64_t end, const uint8_t* alive,
                                                uint64_t amask, uint32_t step, bool photon,
                                                int tid, const RT* s_rad,
                                                const RT* s_pair, SINK& sink,
                                                unsigned long long& c_proc,
                                                unsigned long long& c_ood)
{
    const double dt = A.ph.dt;
    const uint32_t cn = (uint32_t)(end - start);  // chunk-relative offsets, as in bulk_kernel
    for (uint64_t base = start; base < end; base += 2 * STEP_BLOCK) {
        uint64_t ii[2], quid[2];
        uint32_t oo[2];
        uint8_t al[2];
        double px[2], py[2], pz[2], wa[2], wp[2], tau0[2];
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            ii[u] = base + (uint64_t)(u * STEP_BLOCK + tid);
            oo[u] = (uint32_t)(base - start) + (uint32_t)(u * STEP_BLOCK + tid);
            const uint32_t oj = min(oo[u], cn - 1u), ob = oj * 8u;
            al[u] = ld_off(alive + (start & amask), oj & (uint32_t)amask);
            px[u] = ld_off(T.px + start, ob);
            py[u] = ld_off(T.py + start, ob);
            pz[u] = ld_off(T.pz + start, ob);
            wa[u] = ld_off(WV.amp + start, ob);
            wp[u] = ld_off(WV.phase + start, ob);
            quid[u] = 0;
            tau0[u] = 0.0;
            if (LOCAL) quid[u] = ld_off(T.uid + start, ob);
            else tau0[u] = ld_off(T.tau + start, ob);
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const uint64_t i = ii[u];
            const bool live = i < end && al[u] != 0;
            double ex, ey, ez, bx, by, bz;
            double qx = px[u], qy = py[u], qz = pz[u];
            plane_wave_fields(WV, wa[u], wp[u], ex, ey, ez, bx, by, bz);
            const bool pushed = PUSH && !photon;
            if (pushed && live) {  // dead slots keep (and write back) their momentum
                const double hq = (T.species == SFQ_POSITRON ? 0.5 : -0.5) * dt;
                boris_push(hq, ex, ey, ez, bx, by, bz, qx, qy, qz);
            }
            double gamma, chi;
            bool ood = false;
            gamma_chi(photon, qx, qy, qz, ex, ey, ez, bx, by, bz, A.ph.lc_over_lr, gamma, chi);
            const double W = photon ? rate_photon<MIXED>(s_pair, A.ph, gamma, chi, &ood)
                                    : rate_lepton<MIXED>(s_rad, A.ph, gamma, chi, &ood);
            bool emit;
            if (!LOCAL) {
                const double tau = tau0[u] - W * dt;
                emit = live && tau < 0.0;
                if (oo[u] < cn) st_off(T.tau + start, oo[u] * 8u, live ? tau : tau0[u]);  // whole lines
            } else {
                const Draw d = philox_draw(A.seed, quid[u], step, SFQ_P_LOCAL);
                emit = live && W * dt > uniform53(d.a);
            }
            if (pushed && oo[u] < cn) {
                st_off(T.px + start, oo[u] * 8u, qx); st_off(T.py + start, oo[u] * 8u, qy);
                st_off(T.pz + start, oo[u] * 8u, qz);
            }
            if (live) {
                ++c_proc;
                if (T.chi_out) T.chi_out[i] = chi;
                if (T.rate_out) T.rate_out[i] = W;
                c_ood += ood ? 1 : 0;
            }
            EmitRec er;
            er.i = (uint32_t)i;
            er.chi = chi; er.gamma = gamma;
            er.px = qx; er.py = qy; er.pz = qz;
            er.uid = quid[u];
            er.aux = 0.0; er.aux2 = 0.0;
            sink.template put<LOCAL>(A, emit, photon, false, t, er);
        }
    }
}

typedef double dv2 __attribute__((ext_vector_type(2)));

// LCFA chunks of array tiles (optical-depth decisions), two adjacent particles per lane per
// iteration: every array is read and the optical depths (and, with the fused push, the pushed
// momenta) written with 16-byte accesses
// (the caller checks the alignment), and each lane carries two independent chains of
// arithmetic, which hides more of their latency at the same number of waves and memory
// streams.  Whole iterations of 2 x STEP_BLOCK particles only; returns how many particles of the
// chunk it took (the one-particle loop does the rest).  The arithmetic is bulk_kernel's.
template <bool MIXED, bool PUSH, typename SINK, typename RT>
__device__ __forceinline__ uint32_t lcfa_array_vec2(const StepArgs& A, const sfq_tile& T, int t,
                                                    uint64_t start, uint64_t end,
                                                    const uint8_t* alive, uint64_t amask,
                                                    bool photon, int tid,
                                                    const RT* s_rad, const RT* s_pair,
                                                    SINK& sink, unsigned long long& c_proc,
                                                    unsigned long long& c_ood)
{
    const double dt = A.ph.dt;
    const uint32_t cn = (uint32_t)(end - start);
    const uint32_t full = cn - cn % (2u * STEP_BLOCK);
    for (uint32_t ob0 = 0; ob0 < full; ob0 += 2u * STEP_BLOCK) {
        const uint32_t o = ob0 + 2u * (uint32_t)tid;   // even: particles o, o + 1
        const uint32_t ob = o * 8u;
        uint16_t al2 = 0x0101;
        if (amask) al2 = ld_off((const uint16_t*)(alive + start), o);
        const dv2 px = ld_off((const dv2*)(T.px + start), ob);
        const dv2 py = ld_off((const dv2*)(T.py + start), ob);
        const dv2 pz = ld_off((const dv2*)(T.pz + start), ob);
        const dv2 ex = ld_off((const dv2*)(T.ex + start), ob);
        const dv2 ey = ld_off((const dv2*)(T.ey + start), ob);
        const dv2 ez = ld_off((const dv2*)(T.ez + start), ob);
        const dv2 bx = ld_off((const dv2*)(T.bx + start), ob);
        const dv2 by = ld_off((const dv2*)(T.by + start), ob);
        const dv2 bz = ld_off((const dv2*)(T.bz + start), ob);
        const dv2 t0 = ld_off((const dv2*)(T.tau + start), ob);
        __builtin_amdgcn_sched_barrier(0);
        dv2 tout, qxo, qyo, qzo;
        bool em[2];
        double chiv[2], gamv[2];
        const bool pushed = PUSH && !photon;
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const bool live = ((al2 >> (8 * u)) & 0xff) != 0;
            double qx = px[u], qy = py[u], qz = pz[u];
            if (pushed && live) {  // dead slots keep (and write back) their momentum
                const double hq = (T.species == SFQ_POSITRON ? 0.5 : -0.5) * dt;
                boris_push(hq, ex[u], ey[u], ez[u], bx[u], by[u], bz[u], qx, qy, qz);
            }
            qxo[u] = qx; qyo[u] = qy; qzo[u] = qz;
            double gamma, chi;
            bool ood = false;
            gamma_chi(photon, qx, qy, qz, ex[u], ey[u], ez[u], bx[u], by[u], bz[u],
                      A.ph.lc_over_lr, gamma, chi);
            const double W = photon ? rate_photon<MIXED>(s_pair, A.ph, gamma, chi, &ood)
                                    : rate_lepton<MIXED>(s_rad, A.ph, gamma, chi, &ood);
            const double tau = t0[u] - W * dt;
            em[u] = live && tau < 0.0;
            tout[u] = live ? tau : t0[u];
            chiv[u] = chi; gamv[u] = gamma;
            if (live) {
                ++c_proc;
                const uint64_t i = start + o + u;
                if (T.chi_out) T.chi_out[i] = chi;
                if (T.rate_out) T.rate_out[i] = W;
                c_ood += ood ? 1 : 0;
            }
        }
        if (pushed) {
            st_off((dv2*)(T.px + start), ob, qxo);
            st_off((dv2*)(T.py + start), ob, qyo);
            st_off((dv2*)(T.pz + start), ob, qzo);
        }
        st_off((dv2*)(T.tau + start), ob, tout);
        // compaction of both particles in index order (lane l holds particles 2l, 2l + 1)
        EmitRec er[2];
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            er[u].i = (uint32_t)(start + o + u);
            er[u].chi = chiv[u]; er[u].gamma = gamv[u];
            er[u].px = qxo[u]; er[u].py = qyo[u]; er[u].pz = qzo[u];
            er[u].uid = 0; er[u].aux = 0.0; er[u].aux2 = 0.0;
        }
        sink.put2(A, em, photon, t, er);
    }
    return full;
}

// One wave's share of chunk c (lanes tid = 64 w .. 64 w + 63 of the 256-thread layout).
template <bool MIXED, bool BLCFA, bool LOCAL, bool PUSH, bool WAVE, typename SINK, typename RT>
__device__ __forceinline__ void stream_chunk(const StepArgs& A, int c, int tid, const RT* s_rad,
                                             const RT* s_pair, SINK& sink,
                                             unsigned long long& c_proc,
                                             unsigned long long& c_ood, uint32_t base_step)
{
    static_assert(LOCAL || !BLCFA, "beyond-LCFA steps use local decisions");
    const double dt = A.ph.dt;
    const double idt = 1.0 / dt, idt2 = idt * idt;  // beyond-LCFA finite differences
    const int t = __builtin_amdgcn_readfirstlane(find_tile(A.chunk_off, A.ntiles, c));
    const sfq_tile T = uniform_tile(A.tiles[t]);
    const uint32_t step = base_step + (uint32_t)T.step_offset;
    const uint64_t start = (uint64_t)(c - (int)A.chunk_off[t]) * (uint64_t)A.chunk;
    const uint64_t end = min(start + (uint64_t)A.chunk, T.n);
    const bool photon = (T.species == SFQ_PHOTON);
    const bool blcfa = BLCFA && !photon;
    // tiles without an alive array read a constant 1 instead (no branch)
    const uint8_t* alive = T.alive ? T.alive : k_alive_one;
    const uint64_t amask = T.alive ? ~0ull : 0ull;
    // uniform fields: every lane reads element 0 (one cache line for the wave); a plane
    // wave: the fields are computed from two loaded values per particle
    const uint64_t fmask = T.field_mode == SFQ_FIELDS_UNIFORM ? 0ull : ~0ull;
    const bool wave = WAVE && T.field_mode == SFQ_FIELDS_PLANE_WAVE;
    Wave WV{};
    if (WAVE) WV = uniform_wave(A.tiles[t]);
    // Every lane issues every load of an iteration in one group, the alive flag included
    // (lanes past the end of the chunk read its last particle and drop the result): one
    // memory round trip per iteration, with no load behind a data-dependent branch.  The
    // price is reading the fields of dead particles.
    if constexpr (!BLCFA && WAVE) {
        // LCFA chunks of plane-wave tiles read 16 B of fields per particle instead of 48,
        // so one particle per lane leaves too few bytes in flight to cover HBM latency:
        // every lane takes two particles per iteration, all loads in one group.
        if (wave) {
            lcfa_wave_pairs<MIXED, LOCAL, PUSH>(A, T, WV, t, start, end, alive, amask, step,
                                                photon, tid, s_rad, s_pair, sink, c_proc,
                                                c_ood);
            return;
        }
    }
    const uint32_t cn = (uint32_t)(end - start);  // chunk-relative offsets below
    uint64_t first = start;
    if constexpr (!BLCFA && !LOCAL && !WAVE) {
        // array tiles whose arrays allow 16-byte accesses at the chunk (and 2-byte ones for
        // the alive flags): two adjacent particles per lane (not in the kernels that also
        // take plane-wave tiles, whose register budget the plane-wave loop needs)
        const uintptr_t a16 = (uintptr_t)(T.px + start) | (uintptr_t)(T.py + start) |
                              (uintptr_t)(T.pz + start) | (uintptr_t)(T.ex + start) |
                              (uintptr_t)(T.ey + start) | (uintptr_t)(T.ez + start) |
                              (uintptr_t)(T.bx + start) | (uintptr_t)(T.by + start) |
                              (uintptr_t)(T.bz + start) | (uintptr_t)(T.tau + start);
        const uintptr_t a2 = amask ? (uintptr_t)(alive + start) : 0;
        if (fmask == ~0ull && (a16 & 15) == 0 && (a2 & 1) == 0)
            first += lcfa_array_vec2<MIXED, PUSH>(A, T, t, start, end, alive, amask, photon, tid,
                                                  s_rad, s_pair, sink, c_proc, c_ood);
    }
    for (uint64_t base = first; base < end; base += STEP_BLOCK) {
        const uint64_t i = base + tid;
        const uint64_t j = min(i, end - 1);
        const uint32_t o = (uint32_t)(base - start) + (uint32_t)tid;  // i - start
        const uint32_t oj = min(o, cn - 1u), ob = oj * 8u;               // j - start, bytes
        const uint8_t al = ld_off(alive + (start & amask), oj & (uint32_t)amask);
        bool live = false, emit = false;
        double chi = 0.0, gamma = 0.0, aux = 0.0, aux2 = 0.0, qx = 0.0, qy = 0.0, qz = 0.0;
        uint64_t quid = 0;
        bool ood = false;
        double W = 0.0;
        if (BLCFA) {
            // One load group for both species of a beyond-LCFA step.  Without the push, six
            // slots hold E and B on photon chunks and p^{(n-1/2)}, F_perp on lepton chunks;
            // the lepton-only Delta F and flag slots re-read the momentum and alive flag on
            // photon chunks.  With the push every chunk reads E and B, the tile's momentum
            // is p^{(n-1/2)}, and lepton chunks read F_perp and Delta F in six more slots.
            // (chunk-relative: each slot's array is addressed from the chunk's first element)
            const uint64_t n = T.n;
            const uint64_t m05 = (blcfa && !PUSH) ? ~0ull : fmask;  // slots 0..5
            const uint64_t s05 = start & m05;
            const uint32_t ob05 = ob & (uint32_t)m05;
            const bool wave_f = wave && !(blcfa && !PUSH);  // slots 0..5 hold a plane wave
            const double* q0 = (blcfa && !PUSH) ? T.px_prev : T.ex;
            const double* q1 = (blcfa && !PUSH) ? T.py_prev : T.ey;
            const double* q2 = (blcfa && !PUSH) ? T.pz_prev : T.ez;
            const double* q3 = (blcfa && !PUSH) ? T.fperp : T.bx;
            const double* q4 = (blcfa && !PUSH) ? T.fperp + n : T.by;
            const double* q5 = (blcfa && !PUSH) ? T.fperp + 2 * n : T.bz;
            const double* q6 = blcfa ? T.dfperp : T.px;
            const double* q7 = blcfa ? T.dfperp + n : T.py;
            const double* q8 = blcfa ? T.dfperp + 2 * n : T.pz;
            const uint8_t* q9 = blcfa ? T.just_created + start : alive + (start & amask);
            const uint32_t o9 = blcfa ? oj : (oj & (uint32_t)amask);
            const double* q10 = blcfa ? T.fperp : T.px;
            const double* q11 = blcfa ? T.fperp + n : T.py;
            const double* q12 = blcfa ? T.fperp + 2 * n : T.pz;
            double ux = ld_off(T.px + start, ob), uy = ld_off(T.py + start, ob),
                   uz = ld_off(T.pz + start, ob);
            double a0, a1, a2 = 0.0, a3 = 0.0, a4 = 0.0, a5 = 0.0;
            if (wave_f) {
                a0 = ld_off(WV.amp + start, ob);
                a1 = ld_off(WV.phase + start, ob);
            } else {
                a0 = ld_off(q0 + s05, ob05); a1 = ld_off(q1 + s05, ob05);
                a2 = ld_off(q2 + s05, ob05); a3 = ld_off(q3 + s05, ob05);
                a4 = ld_off(q4 + s05, ob05); a5 = ld_off(q5 + s05, ob05);
            }
            const double rx = ld_off(q6 + start, ob), ry = ld_off(q7 + start, ob),
                         rz = ld_off(q8 + start, ob);
            double o0 = 0.0, o1 = 0.0, o2 = 0.0;
            if (PUSH) {
                o0 = ld_off(q10 + start, ob);
                o1 = ld_off(q11 + start, ob);
                o2 = ld_off(q12 + start, ob);
            }
            const bool fresh = ld_off(q9, o9) != 0;
            quid = ld_off(T.uid + start, ob);
            __builtin_amdgcn_sched_barrier(0);
            live = i < end && al != 0;
            if (wave_f) plane_wave_fields(WV, a0, a1, a0, a1, a2, a3, a4, a5);
            // p^{(n-1/2)} and F_perp^{(n-1)}: loaded, or (with the push) the tile's momentum
            // before the push and the six extra slots
            double vx, vy, vz, ox, oy, oz;
            if (PUSH) {
                vx = ux; vy = uy; vz = uz;
                ox = o0; oy = o1; oz = o2;
                if (blcfa && live) {  // dead slots keep (and write back) their momentum
                    const double hq = (T.species == SFQ_POSITRON ? 0.5 : -0.5) * dt;
                    boris_push(hq, a0, a1, a2, a3, a4, a5, ux, uy, uz);
                }
            } else {
                vx = a0; vy = a1; vz = a2;
                ox = a3; oy = a4; oz = a5;
            }
            qx = ux; qy = uy; qz = uz;
            if (!blcfa) {
                gamma_chi(true, ux, uy, uz, a0, a1, a2, a3, a4, a5, A.ph.lc_over_lr, gamma, chi);
                W = rate_photon<MIXED>(s_pair, A.ph, gamma, chi, &ood);
                const Draw d = philox_draw(A.seed, quid, step, SFQ_P_LOCAL);
                emit = live && W * dt > uniform53(d.a);
            } else {
                // beyond-LCFA force update, Sec. 5 Eqs. (fl)-(condit)
                const double flx = (ux - vx) * idt, fly = (uy - vy) * idt, flz = (uz - vz) * idt;
                const double plx = 0.5 * (ux + vx), ply = 0.5 * (uy + vy), plz = 0.5 * (uz + vz);
                const double g2 = 1.0 + (plx * plx + ply * ply + plz * plz);
                gamma = sqrt_nr(g2);
                const double fp = (flx * plx + fly * ply + flz * plz) * rcp_nr(g2);
                const double Fx = flx - fp * plx, Fy = fly - fp * ply, Fz = flz - fp * plz;
                const double F2 = Fx * Fx + Fy * Fy + Fz * Fz;
                const double tc = A.ph.lc_over_lr;
                chi = tc * gamma * sqrt(F2);
                W = rate_lepton<MIXED>(s_rad, A.ph, gamma, chi, &ood);
                if (live) {
                    st_off(T.fperp + start, o * 8u, Fx); st_off(T.fperp + n + start, o * 8u, Fy);
                    st_off(T.fperp + 2 * n + start, o * 8u, Fz);
                }
                if (live && fresh) {
                    st_off(T.dfperp + start, o * 8u, 0.0);
                    st_off(T.dfperp + n + start, o * 8u, 0.0);
                    st_off(T.dfperp + 2 * n + start, o * 8u, 0.0);
                    st_off(T.just_created + start, o, (uint8_t)0);
                } else if (live) {
                    const double ax = Fx - ox, ay = Fy - oy, az = Fz - oz;
                    const double d1x = ax * idt, d1y = ay * idt, d1z = az * idt;
                    const double d2x = (ax - rx) * idt2, d2y = (ay - ry) * idt2, d2z = (az - rz) * idt2;
                    const double delta = tc * tc * ((d1x * d1x + d1y * d1y + d1z * d1z) +
                                                    fabs(Fx * d2x + Fy * d2y + Fz * d2z));
                    st_off(T.dfperp + start, o * 8u, ax);
                    st_off(T.dfperp + n + start, o * 8u, ay);
                    st_off(T.dfperp + 2 * n + start, o * 8u, az);
                    const bool flag = (g2 * delta / (ZETA * ZETA) > chi * chi * F2) && (chi > ZETA);
                    const Draw d = philox_draw(A.seed, quid, step, SFQ_P_LOCAL);
                    emit = W * dt > uniform53(d.a);
                    if (emit) {
                        // energy of the pushed momentum minus gamma^{(n)} (for the recoil)
                        const double pu2 = ux * ux + uy * uy + uz * uz;
                        aux2 = (pu2 - (g2 - 1.0)) / (sqrt(1.0 + pu2) + gamma);
                        // tau / tau_C of Sec. 5 for the threshold gamma_{gamma,LCFA}, which
                        // the emitter pass evaluates (only emitting lanes pay for its
                        // transcendentals there); a negative value: LCFA throughout
                        if (flag) {
                            aux = 2.0 * PI * sqrt(F2 / delta);
                        } else if (chi > ZETA) {
                            aux = -1.0;  // fields effectively constant
                        } else {
                            emit = false;
                        }
                    }
                }
                // the pushed momentum of every slot of the chunk, so that whole cache lines
                // are written (emitters get theirs again in the emitter pass, after the
                // recoil or the rejection; dead slots write back their own)
                if (PUSH && i < end) {
                    st_off(T.px + start, o * 8u, ux); st_off(T.py + start, o * 8u, uy);
                    st_off(T.pz + start, o * 8u, uz);
                }
            }
        } else {
            qx = ld_off(T.px + start, ob); qy = ld_off(T.py + start, ob);
            qz = ld_off(T.pz + start, ob);
            const uint64_t fs = start & fmask;         // uniform fields: element 0
            const uint32_t obf = ob & (uint32_t)fmask;
            double ex, ey, ez = 0.0, bx = 0.0, by = 0.0, bz = 0.0;
            if (wave) {
                ex = ld_off(WV.amp + start, ob);
                ey = ld_off(WV.phase + start, ob);
            } else {
                ex = ld_off(T.ex + fs, obf); ey = ld_off(T.ey + fs, obf);
                ez = ld_off(T.ez + fs, obf); bx = ld_off(T.bx + fs, obf);
                by = ld_off(T.by + fs, obf); bz = ld_off(T.bz + fs, obf);
            }
            double tau0 = 0.0;
            if (LOCAL) quid = ld_off(T.uid + start, ob);
            else tau0 = ld_off(T.tau + start, ob);
            // keep the whole load group ahead of the arithmetic: the first use of a loaded
            // value waits for every outstanding memory operation (loads and stores share
            // one counter here), so a use scheduled between the loads would split the group
            __builtin_amdgcn_sched_barrier(0);
            live = i < end && al != 0;
            if (wave) plane_wave_fields(WV, ex, ey, ex, ey, ez, bx, by, bz);
            const bool pushed = PUSH && !photon;
            if (pushed && live) {  // dead slots keep (and write back) their momentum
                const double hq = (T.species == SFQ_POSITRON ? 0.5 : -0.5) * dt;
                boris_push(hq, ex, ey, ez, bx, by, bz, qx, qy, qz);
            }
            gamma_chi(photon, qx, qy, qz, ex, ey, ez, bx, by, bz, A.ph.lc_over_lr, gamma, chi);
            W = photon ? rate_photon<MIXED>(s_pair, A.ph, gamma, chi, &ood)
                       : rate_lepton<MIXED>(s_rad, A.ph, gamma, chi, &ood);
            if (!LOCAL) {
                const double tau = tau0 - W * dt;
                emit = live && tau < 0.0;
                // Every slot of the chunk is written, dead ones with their own value: a
                // partly written cache line costs the memory a read-modify-write.  Emitters
                // get a fresh depth in the emitter pass; a converting photon keeps the
                // decremented one.
                if (o < cn) st_off(T.tau + start, o * 8u, live ? tau : tau0);
            } else {
                const Draw d = philox_draw(A.seed, quid, step, SFQ_P_LOCAL);
                emit = live && W * dt > uniform53(d.a);
            }
            // the pushed momentum of every slot (whole cache lines, as for tau): emitters
            // recoil from the queued, pushed momentum in the emitter pass, which then
            // overwrites it
            if (pushed && o < cn) {
                st_off(T.px + start, o * 8u, qx); st_off(T.py + start, o * 8u, qy);
                st_off(T.pz + start, o * 8u, qz);
            }
        }
        if (live) {
            ++c_proc;
            if (T.chi_out) T.chi_out[i] = chi;
            if (T.rate_out) T.rate_out[i] = W;
            c_ood += ood ? 1 : 0;
        }
        // compaction: the whole iteration is one tile, hence one species
        EmitRec er;
        er.i = (uint32_t)i;
        er.chi = chi; er.gamma = gamma;
        er.px = qx; er.py = qy; er.pz = qz;
        er.uid = quid;
        er.aux = aux; er.aux2 = aux2;
        sink.template put<LOCAL>(A, emit, photon, blcfa, t, er);
    }
}

// The streaming work of block b of G: its waves' queue slices are STEP_WAVES b ... .  Chunks
// are taken one at a time from a step-wide counter (the next one fetched while the current one
// streams), at most A.max_chunks per block: blocks that start late or run slow take fewer, so
// the grid finishes together instead of waiting for its slowest block's fixed share.  (Which
// block streams a chunk changes no result, only the order of products in their buffers.)
// s_tmp: two words of shared memory.
template <bool MIXED, bool BLCFA, bool LOCAL, bool PUSH, bool WAVE, typename RT>
__device__ __forceinline__ void stream_block(const StepArgs& A, int b, int G, RT* s_rad,
                                             RT* s_pair, unsigned long long* s_cnt,
                                             unsigned long long* s_tmp)
{
    static_assert(LOCAL || !BLCFA, "beyond-LCFA steps use local decisions");
    const int tid = threadIdx.x;
    const RT* g_rad = MIXED ? (const RT*)A.tb.rad32 : (const RT*)A.tb.rad;
    const RT* g_pair = MIXED ? (const RT*)A.tb.pair32 : (const RT*)A.tb.pair;
    for (int k = tid; k < RAD_SIZE; k += STEP_BLOCK) s_rad[k] = g_rad[k];
    for (int k = tid; k < PAIR_SIZE; k += STEP_BLOCK) s_pair[k] = g_pair[k];
    if (tid < CNT_N) s_cnt[tid] = 0;
    // beyond-LCFA photons take their slots by atomics in the emitter kernel: a step whose
    // product counts start from zero starts that count here
    if (BLCFA && A.zero_counts && A.nsets == 0 && b == 0 && tid == 0) A.prod_counts[0] = 0;
    __syncthreads();

    unsigned long long c_proc = 0, c_ood = 0;
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    const uint64_t slice = (uint64_t)b * STEP_WAVES + (uint64_t)wv;
    QueueSink sink{slice * A.q_cap_per_wave, 0u, 0u};
    const uint32_t share = (uint32_t)(A.chunk / STEP_WAVES);  // most particles of a wave's share
    const uint32_t base_step = A.step_ptr ? (uint32_t)*A.step_ptr : A.step;

    // every chunk index the counter hands out below N is streamed (or deferred) by the block
    // that got it; G blocks of at most max_chunks >= ceil(N / G) each take all N
    __shared__ int s_chunk;
    if (tid == 0) s_chunk = (int)atomicAdd(&A.d_ctl[4], 1u);
    __syncthreads();
    int c = s_chunk, taken = 0;
    for (; c < A.nchunks && taken < A.max_chunks; ++taken) {
        unsigned nxt = 0;
        if (tid == 0 && taken + 1 < A.max_chunks) nxt = atomicAdd(&A.d_ctl[4], 1u);
        // a share whose every particle might emit must fit the slice; otherwise it is left
        // untouched for the deferred-share kernel (no result depends on which wave steps it)
        if (A.q_cap_per_wave - (uint64_t)(sink.nl + sink.np) < (uint64_t)share) {
            if (lane_id() == 0) {
                const unsigned k = atomicAdd(&A.d_ctl[0], 1u);
                A.d_list[k] = (uint32_t)c * STEP_WAVES + (uint32_t)wv;
            }
        } else {
            stream_chunk<MIXED, BLCFA, LOCAL, PUSH, WAVE>(A, c, tid, s_rad, s_pair, sink, c_proc,
                                                           c_ood, base_step);
        }
        __syncthreads();  // every wave is done with s_chunk
        if (tid == 0) s_chunk = taken + 1 < A.max_chunks ? (int)nxt : A.nchunks;
        __syncthreads();
        c = s_chunk;
    }
    if (lane_id() == 0) {
        A.q_count[2 * slice] = sink.nl;
        A.q_count[2 * slice + 1] = sink.np;
    }
    // the block's totals (what the emitter kernel sums over earlier blocks) and the block's
    // processed count go to the queue for the emitter kernel (no global atomic:
    // thousands of blocks adding to one word serialise); the rare out-of-domain count is added
    unsigned long long tl = lane_id() == 0 ? sink.nl : 0u, tp = lane_id() == 0 ? sink.np : 0u;
    block_sum2(s_tmp, tl, tp);
    const unsigned long long proc = block_sum(s_tmp, c_proc);
    if (tid == 0) {
        reinterpret_cast<uint4*>(A.q_sbcount)[b] = make_uint4((uint32_t)tl, (uint32_t)tp,
                                                               (uint32_t)taken, 0u);
        A.q_proc[b] = proc;
    }
    const unsigned long long vals[CNT_N] = {0, 0, 0, 0, c_ood, 0, 0, 0};
    block_add_counters(s_cnt, A.counters, vals);
}

template <bool MIXED, bool BLCFA, bool LOCAL, bool PUSH, bool WAVE>
__global__ __launch_bounds__(STEP_BLOCK, bulk_waves(MIXED, BLCFA, PUSH, WAVE)) void bulk_kernel(StepArgs A)
{
    using RT = typename std::conditional<MIXED, float, double>::type;
    __shared__ RT s_rad[RAD_SIZE];
    __shared__ RT s_pair[PAIR_SIZE];
    __shared__ unsigned long long s_cnt[CNT_N];
    __shared__ unsigned long long s_tmp[2];
    stream_block<MIXED, BLCFA, LOCAL, PUSH, WAVE>(A, (int)blockIdx.x, (int)gridDim.x, s_rad,
                                                   s_pair, s_cnt, s_tmp);
}


// Emitter pass: the slices of streaming block qb are sampled by emit_split blocks with every
// lane busy, each taking a contiguous range of their entries: Philox draws, inverse-CDF tables,
// recoil and products.
// Product slots: every queued lepton emits one photon and every queued photon converts into
// one pair (beyond-LCFA rejections are only known here, so that mode takes photon slots by
// atomics, and steps with per-tile product sets by atomics per set).  A block's slots start at
// the product counts before the step plus the emitters queued by every earlier streaming
// block: each block sums those counts itself (one coalesced read of the per-block totals);
// block 0 adds the step's processed / emitted / converted counters once and the last block out
// advances the product counts, so no scan kernel runs between the two passes.
struct EmitShared {
    unsigned cum[2 * STEP_WAVES + 1];
    unsigned long long base[3 * STEP_WAVES];
    unsigned long long tmp[2];
    uint2 own[STEP_WAVES];
    unsigned long long b[3];
    unsigned chunks;  // chunks streamed by the streaming block
};

// The emitter work of one block (every thread calls it): part `part` of the entries queued by
// streaming block qb.
template <bool MIXED, bool BLCFA, bool LOCAL>
__device__ __forceinline__ void emit_item(const StepArgs& A, int qb, int part, EmitCounts& C,
                                          EmitShared& sh)
{
    static_assert(LOCAL || !BLCFA, "beyond-LCFA steps use local decisions");
    const int tid = threadIdx.x;
    const uint32_t base_step = A.step_ptr ? (uint32_t)*A.step_ptr : A.step;
    const bool multi = A.nsets > 0;
    // zeroed counts: the bases are 0 (no separate zeroing kernel before the step)
    const bool from0 = multi || A.zero_counts;
    const uint2* qc = reinterpret_cast<const uint2*>(A.q_count);
    // the emitters queued by the streaming blocks before qb, qb's own slice counts and the
    // product counts before the step (only the last block out changes them, after every block
    // has read them here): all loads issued together, one memory round trip
    unsigned long long pl = 0, pp = 0;
    {
        const uint4* qs = reinterpret_cast<const uint4*>(A.q_sbcount);
#pragma unroll 4
        for (int k = tid; k < qb; k += STEP_BLOCK) {
            const uint4 c = qs[k];
            pl += c.x;
            pp += c.y;
        }
        const int s_lo = qb * STEP_WAVES;
        if (tid < STEP_WAVES) sh.own[tid] = qc[s_lo + tid];
        else if (tid < STEP_WAVES + 3)
            sh.b[tid - STEP_WAVES] = from0 ? 0ull : A.prod_counts[tid - STEP_WAVES];
        else if (tid == STEP_WAVES + 3)
            sh.chunks = qs[qb].z;
    }
    block_sum2(sh.tmp, pl, pp);  // its barriers also publish sh.own and sh.b
    // qb's slices in order: leptons then photons of slice 0, of slice 1, ...
    if (tid == 0) {
        unsigned acc = 0;
        unsigned long long rl = pl, rp = pp;
        for (int w = 0; w < STEP_WAVES; ++w) {
            const uint2 c = sh.own[w];
            sh.cum[2 * w] = acc;
            acc += c.x;
            sh.cum[2 * w + 1] = acc;
            acc += c.y;
            // this slice's first photon, electron and positron slots
            sh.base[3 * w] = multi ? 0ull : sh.b[0] + rl;
            sh.base[3 * w + 1] = multi ? 0ull : sh.b[1] + rp;
            sh.base[3 * w + 2] = multi ? 0ull : sh.b[2] + rp;
            rl += c.x;
            rp += c.y;
        }
        sh.cum[2 * STEP_WAVES] = acc;
    }
    __syncthreads();
    const unsigned total = sh.cum[2 * STEP_WAVES];
    // where the streaming block found emitters dense, the products are written with
    // non-temporal stores, which are faster there; where they are sparse, ordinary stores are
    // faster (measured at 2 % and 13 % emitters)
    const bool nt_prod =
        (float)total > DENSE_EMITTER_FRACTION * (float)sh.chunks * (float)A.chunk;
    const unsigned per = (total + A.emit_split - 1) / A.emit_split;
    const unsigned e_lo = min(total, per * (unsigned)part), e_hi = min(total, e_lo + per);
    for (unsigned b0e = e_lo; b0e < e_hi; b0e += STEP_BLOCK) {
        const unsigned e = b0e + tid;
        const bool valid = e < e_hi;
        // this lane's entry: the segment (slice, species) that holds entry e
        int k = 0;
#pragma unroll
        for (int j = 1; j < 2 * STEP_WAVES; ++j)
            if (e >= sh.cum[j]) k = j;
        const int w = k >> 1;
        const bool pair = valid && (k & 1);
        const unsigned rank = e - sh.cum[k];
        const uint64_t sbase = ((uint64_t)qb * STEP_WAVES + w) * A.q_cap_per_wave;
        const uint64_t slot = pair ? sbase + A.q_cap_per_wave - 1 - rank : sbase + rank;
        uint32_t i = 0;
        int t = 0;
        double chi = 1.0, gamma = 1.0, px = 0, py = 0, pz = 0, aux = -1.0, aux2 = 0.0;
        uint64_t quid = 0;
        // the entry is read once: non-temporal loads (measured faster, most where emitters are
        // dense)
        if (valid) {
            i = ld_stream(&A.q_idx[slot]);
            t = (int)ld_stream(&A.q_tile[slot]);
            chi = ld_stream(&A.q_chi[slot]);
            gamma = ld_stream(&A.q_gamma[slot]);
            px = ld_stream(&A.q_px[slot]);
            py = ld_stream(&A.q_py[slot]);
            pz = ld_stream(&A.q_pz[slot]);
            if (LOCAL) quid = ld_stream(&A.q_uid[slot]);
            if (BLCFA && !pair) {
                aux = ld_stream(&A.q_aux[slot]);
                aux2 = ld_stream(&A.q_aux2[slot]);
            }
        }
        emit_one<MIXED, BLCFA, LOCAL>(A, valid, pair, i, t, chi, gamma, px, py, pz, quid, aux,
                                      aux2, base_step, false, sh.base[3 * w] + rank,
                                      sh.base[3 * w + 1] + rank, sh.base[3 * w + 2] + rank, C,
                                      nt_prod);
    }
}

template <bool MIXED, bool BLCFA, bool LOCAL>
__global__ __launch_bounds__(STEP_BLOCK, SFQ_EMIT_WAVES) void emit_kernel(StepArgs A)
{
    __shared__ unsigned long long s_cnt[CNT_N];
    __shared__ EmitShared sh;
    __shared__ unsigned s_fmax;
    __shared__ int s_last;
    const int tid = threadIdx.x;
    const bool multi = A.nsets > 0;
    const int G = A.grid;
    if (tid < CNT_N) s_cnt[tid] = 0;
    if (blockIdx.x == 0) {
        // Block 0 first adds the step's processed / emitted / converted counters (every queued
        // lepton emits, every queued photon converts; beyond-LCFA acceptances are counted by
        // the blocks) and stores the observations for sizing the queue: the largest emitter
        // fraction of a wave's shares and the shares deferred (plain stores to host memory,
        // which the host reads at a later step; a late or overwritten value only delays a
        // resize).  All of it comes from what the streaming kernel wrote.
        const uint2* qc = reinterpret_cast<const uint2*>(A.q_count);
        const int S = G * STEP_WAVES;
        unsigned long long tl = 0, tp = 0, proc = 0, dummy = 0;
        float fmax = 0.0f;
        if (tid == 0) s_fmax = 0;
        const uint4* qs = reinterpret_cast<const uint4*>(A.q_sbcount);
#pragma unroll 8
        for (int sl = tid; sl < S; sl += STEP_BLOCK) {
            const uint2 c = qc[sl];
            tl += c.x;
            tp += c.y;
            if (A.obs) {
                // the emitter fraction of the wave's shares: its block's chunks times a share
                const unsigned chunks = qs[sl / STEP_WAVES].z;
                const float room = (float)chunks * (float)(A.chunk / STEP_WAVES);
                if (room > 0.0f) fmax = fmaxf(fmax, (float)(c.x + c.y) / room);
            }
        }
#pragma unroll 4
        for (int b = tid; b < G; b += STEP_BLOCK) proc += A.q_proc[b];
        block_sum2(sh.tmp, tl, tp);  // its first barrier also publishes s_fmax = 0
        if (A.obs && fmax > 0.0f) atomicMax(&s_fmax, __float_as_uint(fmax));  // fmax >= 0
        block_sum2(sh.tmp, proc, dummy);
        if (tid == 0) {
            atomicAdd(&A.counters->processed, proc);
            if (!BLCFA) atomicAdd(&A.counters->emitted, tl);
            atomicAdd(&A.counters->converted, tp);
            if (A.obs) {
                A.obs[0] = s_fmax;
                A.obs[1] = A.d_ctl[0];
            }
            if (A.emit_obs && proc > 0)
                *A.emit_obs = __float_as_uint((float)(tl + tp) / (float)proc);
        }
    }
    EmitCounts C;
    emit_item<MIXED, BLCFA, LOCAL>(A, (int)blockIdx.x / A.emit_split,
                                   (int)blockIdx.x % A.emit_split, C, sh);
    __syncthreads();
    const unsigned long long vals[CNT_N] = {0, BLCFA ? C.emit : 0ull, 0, C.rej, C.ood, C.clamp,
                                            C.over, 0};
    block_add_counters(s_cnt, A.counters, vals);
    // The last block out advances the product counts.  It reads only what the streaming kernel
    // wrote, and every block's read of the product counts returned before its count here, so
    // no memory fence is needed (a device-scope fence would write back the whole L2 of the
    // block's XCD, in every block).
    if (tid == 0) {
        const unsigned done = atomicAdd(&A.d_ctl[3], 1u);
        s_last = done == gridDim.x - 1;
    }
    __syncthreads();
    if (!s_last) return;
    if (!multi) {
        const uint4* qs = reinterpret_cast<const uint4*>(A.q_sbcount);
        unsigned long long tl = 0, tp = 0;
#pragma unroll 4
        for (int b = tid; b < G; b += STEP_BLOCK) {
            const uint4 c = qs[b];
            tl += c.x;
            tp += c.y;
        }
        block_sum2(sh.tmp, tl, tp);
        if (tid == 0) {
            // beyond-LCFA photons took their slots by atomics from this count (which the
            // streaming kernel zeroed when the step starts from zero)
            if (!BLCFA) A.prod_counts[0] = (A.zero_counts ? 0ull : A.prod_counts[0]) + tl;
            A.prod_counts[1] = (A.zero_counts ? 0ull : A.prod_counts[1]) + tp;
            A.prod_counts[2] = (A.zero_counts ? 0ull : A.prod_counts[2]) + tp;
        }
    }
    if (tid == 0) {
        A.d_ctl[3] = 0;
        A.d_ctl[4] = 0;  // the next step's streaming kernel takes chunks from 0 again
    }
}

// The shares the streaming pass deferred (enqueued after the emitter kernel whenever the
// queue is smaller than a step's worst case; it returns at once when nothing was deferred).
// Each wave takes one share at a time and steps it whole: the streaming pass's arithmetic on
// the same inputs (the rate tables read from global memory), each emitter's work done at once
// with product slots taken by atomics.  The last block out clears the deferral words.
template <bool MIXED, bool BLCFA, bool LOCAL, bool PUSH, bool WAVE>
__global__ __launch_bounds__(STEP_BLOCK, 1) void defer_kernel(StepArgs A)
{
    static_assert(LOCAL || !BLCFA, "beyond-LCFA steps use local decisions");
    using RT = typename std::conditional<MIXED, float, double>::type;
    __shared__ unsigned long long s_cnt[CNT_N];
    const unsigned ndef = A.d_ctl[0];
    if (ndef == 0) return;  // the same for every block: nothing to step, nothing to clear
    const int tid = threadIdx.x;
    if (tid < CNT_N) s_cnt[tid] = 0;
    __syncthreads();
    const uint32_t base_step = A.step_ptr ? (uint32_t)*A.step_ptr : A.step;
    const RT* g_rad = MIXED ? (const RT*)A.tb.rad32 : (const RT*)A.tb.rad;
    const RT* g_pair = MIXED ? (const RT*)A.tb.pair32 : (const RT*)A.tb.pair;
    EmitCounts C;
    InlineSink<MIXED, BLCFA, LOCAL> sink{&C, base_step};
    unsigned long long c_proc = 0, c_ood = 0;
    for (;;) {
        unsigned u = 0;
        if (lane_id() == 0) u = atomicAdd(&A.d_ctl[1], 1u);
        u = __shfl(u, 0);
        if (u >= ndef) break;
        const uint32_t unit = A.d_list[u];
        const int c = (int)(unit / STEP_WAVES), wu = (int)(unit % STEP_WAVES);
        stream_chunk<MIXED, BLCFA, LOCAL, PUSH, WAVE>(A, c, wu * 64 + lane_id(), g_rad, g_pair,
                                                       sink, c_proc, c_ood, base_step);
    }
    __syncthreads();
    const unsigned long long vals[CNT_N] = {c_proc, C.emit, C.conv, C.rej, C.ood + c_ood,
                                            C.clamp, C.over, c_proc};
    block_add_counters(s_cnt, A.counters, vals);
    // the last block out clears the deferral words (every block is past its last use of them
    // when it counts itself out; no fence: the next kernel sees the stores)
    if (tid == 0) {
        const unsigned done = atomicAdd(&A.d_ctl[2], 1u);
        if (done == gridDim.x - 1) {
            A.d_ctl[0] = 0;
            A.d_ctl[1] = 0;
            A.d_ctl[2] = 0;
        }
    }
}

// step helpers: zero the product counts of product sets (a kernel, not a memset, so graphs
// replay it safely) and advance a plan's device step counter after a step
__global__ void zero_set_counts_kernel(const sfq_product_set* sets, int nsets)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < 3 * nsets) sets[k / 3].product_counts[k % 3] = 0;
}

__global__ void advance_step_kernel(unsigned long long* step)
{
    if (threadIdx.x == 0) *step += 1;
}

__global__ void set_step_kernel(unsigned long long* step, unsigned long long value)
{
    if (threadIdx.x == 0) *step = value;
}

// =============================================================================================
// Batched elementwise kernels
// =============================================================================================
template <bool MIXED>
__global__ __launch_bounds__(256) void rates_kernel(Tables tb, Physics ph, int photon, size_t n,
                                                    const double* gamma, const double* chi,
                                                    double* out)
{
    using RT = typename std::conditional<MIXED, float, double>::type;
    __shared__ RT s_tab[RAD_SIZE > PAIR_SIZE ? RAD_SIZE : PAIR_SIZE];
    const RT* src = photon ? (MIXED ? (const RT*)tb.pair32 : (const RT*)tb.pair)
                           : (MIXED ? (const RT*)tb.rad32 : (const RT*)tb.rad);
    const int sz = photon ? PAIR_SIZE : RAD_SIZE;
    for (int k = threadIdx.x; k < sz; k += blockDim.x) s_tab[k] = src[k];
    __syncthreads();
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x) {
        bool ood = false;
        out[i] = photon ? rate_photon<MIXED>(s_tab, ph, gamma[i], chi[i], &ood)
                        : rate_lepton<MIXED>(s_tab, ph, gamma[i], chi[i], &ood);
    }
}

__global__ __launch_bounds__(256) void chi_kernel(int photon, size_t n, const double* px,
                                                  const double* py, const double* pz,
                                                  const double* ex, const double* ey,
                                                  const double* ez, const double* bx,
                                                  const double* by, const double* bz,
                                                  double lc, double* gamma_out, double* chi_out)
{
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x) {
        double g, c;
        gamma_chi(photon != 0, px[i], py[i], pz[i], ex[i], ey[i], ez[i], bx[i], by[i], bz[i], lc,
                  g, c);
        if (gamma_out) gamma_out[i] = g;
        chi_out[i] = c;
    }
}

// uniform loops: every lane of a wave takes part in the cooperative table evaluation
template <bool MIXED>
__global__ __launch_bounds__(256) void sample_photon_kernel(Tables tb, size_t n,
                                                            const double* gamma,
                                                            const double* chi, const double* r,
                                                            double* gph, double* gem)
{
    for (size_t base = blockIdx.x * (size_t)blockDim.x; base < n;
         base += (size_t)gridDim.x * blockDim.x) {
        const size_t i = base + threadIdx.x;
        const bool valid = i < n;
        double s = 0, v, omv;
        bool ood;
        sample_coop<MIXED>(tb, valid, false, valid ? chi[i] : 1.0, valid ? r[i] : 0.5, s, v, omv,
                           ood);
        if (valid) {
            const double g = gamma[i];
            gph[i] = g * (s / (1.0 + s));
            if (gem) gem[i] = g / (1.0 + s);
        }
    }
}

template <bool MIXED>
__global__ __launch_bounds__(256) void sample_pair_kernel(Tables tb, size_t n, const double* gamma,
                                                          const double* chi, const double* r,
                                                          double* ge, double* gp)
{
    for (size_t base = blockIdx.x * (size_t)blockDim.x; base < n;
         base += (size_t)gridDim.x * blockDim.x) {
        const size_t i = base + threadIdx.x;
        const bool valid = i < n;
        double s, v = 0, omv = 1;
        bool ood;
        const double ri = valid ? r[i] : 0.5;
        sample_coop<MIXED>(tb, valid, true, valid ? chi[i] : 1.0, ri, s, v, omv, ood);
        if (valid) {
            double a, b;
            pair_energies(gamma[i], ri, v, omv, a, b);
            ge[i] = a;
            if (gp) gp[i] = b;
        }
    }
}

__global__ __launch_bounds__(256) void philox_kernel(size_t n, const uint64_t* uid, uint64_t seed,
                                                     uint32_t step, uint32_t purpose,
                                                     uint64_t* a, uint64_t* b)
{
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x) {
        const Draw d = philox_draw(seed, uid[i], step, purpose);
        a[i] = d.a;
        if (b) b[i] = d.b;
    }
}

__global__ __launch_bounds__(256) void init_tau_kernel(size_t n, const uint64_t* uid,
                                                       uint64_t seed, double* tau)
{
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        tau[i] = optical_depth(philox_draw(seed, uid[i], 0, SFQ_P_INIT).a);
}

// =============================================================================================
// Host side
// =============================================================================================
namespace {

thread_local std::string tl_error = "";

struct Staging {
    void* host = nullptr;   // pinned
    void* dev = nullptr;
    hipEvent_t done = nullptr;
    size_t bytes = 0;
};

constexpr int N_STAGING = 8;
constexpr size_t STAGING_BYTES = 2 << 20;

}  // namespace

// Scratch of the step that allocates nothing (sfq_step_noalloc): the tile descriptors (the first
// STAGING_BYTES), then the emitter queue and the deferred-share list, in a file-scope device
// array of fixed size.  Each device holds its own copy until the process ends; host code uses
// its device address, queried once per device at set-up (the array's name is not a device
// address in host code).
constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)256 << 20;
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

namespace {
std::mutex g_scratch_mu;
std::vector<void*> g_scratch_ptr;  // by device ordinal
}  // namespace

struct ProfEvents {
    hipEvent_t e[3];
    int split;  // e[1] recorded between the streaming kernel and the emitter pass
};

struct sfq_ctx {
    int device = 0;
    int precision = SFQ_FP64, decision = SFQ_OPTICAL_DEPTH, blcfa = 0, bw_fast = 0;
    int approx = SFQ_APPROX_FULL;
    double lc_over_lr = 0, lr_over_lc = 0, dt = 0;
    Physics ph{};
    Tables tb{};
    void* d_tab64 = nullptr;
    void* d_tab32 = nullptr;
    int num_cus = 256;
    // step scratch: the emitter queue and its capacities (entries, slices, blocks, deferrable
    // shares), and its sizing: room for q_frac of a wave's particles beyond one share, grown
    // from what the steps observe when q_adaptive
    std::mutex mu;
    void* d_queue = nullptr;
    uint64_t q_cap_entries = 0, q_cap_slices = 0, q_cap_grid = 0, q_cap_deferrable = 0;
    double q_frac = 0.125;
    int q_adaptive = 1;
    unsigned* obs_host = nullptr;  // pinned, mapped: the emitter kernel's observations
    unsigned* obs_dev = nullptr;
    double emit_frac = 0.0;        // the emitter fraction of the last step observed (steps and
                                   // plan launches): picks the emitter pass's blocks per CU
    // The end of the handle's last step (its own step_done event, or the step's timing event
    // when timing is on): a step on another stream waits for it, since steps share the queue.
    // One event record per step: a staging slot's event is recorded only when the descriptors
    // move on to another slot (on the stream of the step that moves on, after that wait, so it
    // marks the end of every step that read the slot).
    hipEvent_t step_done = nullptr;
    hipEvent_t last_end = nullptr;
    hipStream_t last_stream = nullptr;
    bool any_step = false;
    Staging staging[N_STAGING];
    int next_staging = 0;
    // the descriptor bytes last uploaded and the staging slot whose device copy holds them: a
    // step with the same descriptors (the same tiles, step after step) reuses that copy
    std::vector<char> last_desc, desc_bytes;
    int last_slot = -1;
    // launch shape of the step kernel (tunable)
    int blocks_per_cu = 8;
    int chunk = 2048;
    // kernel timing (sfq_profile_*): events around the two step kernels of each timed step
    int prof = 0;
    std::vector<ProfEvents> prof_used, prof_free;
    // sfq_step_noalloc: the device's static scratch, and a pinned host buffer and its event for
    // uploading the descriptors (all set up by sfq_create; null when that failed)
    void* na_scratch = nullptr;
    void* na_host = nullptr;
    hipEvent_t na_done = nullptr;
};

struct sfq_plan_t;

static sfq_status fail(sfq_ctx* h, sfq_status st, const std::string& msg)
{
    tl_error = msg;
    (void)h;
    return st;
}

#define HIP_TRY(h, expr)                                                                       \
    do {                                                                                       \
        hipError_t e_ = (expr);                                                                \
        if (e_ != hipSuccess)                                                                  \
            return fail(h, SFQ_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_));   \
    } while (0)

static std::string default_tables_path()
{
    Dl_info info;
    if (dladdr((void*)&sfq_create, &info) && info.dli_fname) {
        std::string p(info.dli_fname);
        const size_t s = p.find_last_of('/');
        std::string dir = (s == std::string::npos) ? std::string(".") : p.substr(0, s);
        return dir + "/data/sfq_tables.bin";
    }
    return "data/sfq_tables.bin";
}

static sfq_status load_tables(sfq_ctx* h, const char* path_in)
{
    const std::string path = path_in ? std::string(path_in) : default_tables_path();
    FILE* f = fopen(path.c_str(), "rb");
    if (!f) return fail(h, SFQ_E_TABLES, "cannot open table file " + path);
    std::vector<char> buf;
    {
        fseek(f, 0, SEEK_END);
        const long sz = ftell(f);
        fseek(f, 0, SEEK_SET);
        buf.resize(sz > 0 ? (size_t)sz : 0);
        const size_t got = buf.empty() ? 0 : fread(buf.data(), 1, buf.size(), f);
        fclose(f);
        if (got != buf.size()) return fail(h, SFQ_E_TABLES, "short read on " + path);
    }
    size_t pos = 0;
    auto need = [&](size_t k) { return pos + k <= buf.size(); };
    if (!need(8 + 16) || memcmp(buf.data(), "SFQTAB03", 8) != 0)
        return fail(h, SFQ_E_TABLES, "bad table file magic in " + path);
    pos = 8;
    uint32_t version, narr;
    uint64_t hash;
    memcpy(&version, &buf[pos], 4);
    memcpy(&narr, &buf[pos + 4], 4);
    memcpy(&hash, &buf[pos + 8], 8);
    pos += 16;
    (void)hash;
    const int expect_geom[24] = {RATE_DEG, CHI_OCT_LO, CHI_OCT_HI, N_CHI_SEG, PAIR_OCT_LO,
                                 N_PAIR_SEG, KA_DEG, N_KA, KB_DEG, KB_OCT_LO, KB_OCT_HI, INV_NC,
                                 INV_NR, N_LO_SEG, T_OCT_LO, T_OCT_HI, N_HI_SEG, N_R_SEG, SUB,
                                 INV_CHI_OCT_LO, N_INV_CHI, N_PAIR_INV_CHI, RATE_DEG_TRUNC,
                                 INV_TRUNC};
    if (version != 3 || narr != 6 || !need(sizeof(expect_geom)))
        return fail(h, SFQ_E_TABLES, "unsupported table file version in " + path);
    int geom[24];
    memcpy(geom, &buf[pos], sizeof(geom));
    pos += sizeof(geom);
    for (int k = 0; k < 24; ++k)
        if (geom[k] != expect_geom[k])
            return fail(h, SFQ_E_TABLES, "table geometry mismatch (field " + std::to_string(k) +
                                             ") in " + path + ": rebuild the tables");
    const size_t sizes[6] = {RAD_SIZE, PAIR_SIZE, KA_SIZE, KB_SIZE, PHINV_SIZE, PPINV_SIZE};
    size_t total = 0;
    for (size_t s : sizes) total += s;
    std::vector<double> host64(total);
    size_t o = 0;
    for (int a = 0; a < 6; ++a) {
        uint64_t cnt;
        if (!need(8)) return fail(h, SFQ_E_TABLES, "truncated table file " + path);
        memcpy(&cnt, &buf[pos], 8);
        pos += 8;
        if (cnt != sizes[a] || !need(cnt * 8))
            return fail(h, SFQ_E_TABLES, "table array size mismatch in " + path);
        memcpy(&host64[o], &buf[pos], cnt * 8);
        pos += cnt * 8;
        o += cnt;
    }
    std::vector<float> host32(total);
    for (size_t k = 0; k < total; ++k) host32[k] = (float)host64[k];
    HIP_TRY(h, hipMalloc(&h->d_tab64, total * sizeof(double)));
    HIP_TRY(h, hipMalloc(&h->d_tab32, total * sizeof(float)));
    HIP_TRY(h, hipMemcpy(h->d_tab64, host64.data(), total * sizeof(double), hipMemcpyHostToDevice));
    HIP_TRY(h, hipMemcpy(h->d_tab32, host32.data(), total * sizeof(float), hipMemcpyHostToDevice));
    const double* d = (const double*)h->d_tab64;
    const float* s = (const float*)h->d_tab32;
    size_t off[6];
    off[0] = 0;
    for (int a = 1; a < 6; ++a) off[a] = off[a - 1] + sizes[a - 1];
    h->tb.rad = d + off[0];
    h->tb.pair = d + off[1];
    h->tb.ka = d + off[2];
    h->tb.kb = d + off[3];
    h->tb.phinv = d + off[4];
    h->tb.ppinv = d + off[5];
    h->tb.rad32 = s + off[0];
    h->tb.pair32 = s + off[1];
    h->tb.phinv32 = s + off[4];
    h->tb.ppinv32 = s + off[5];
    return SFQ_OK;
}

static void release(sfq_ctx* h)
{
    if (!h) return;
    (void)hipSetDevice(h->device);
    for (auto& s : h->staging) {
        if (s.done) {
            (void)hipEventSynchronize(s.done);
            (void)hipEventDestroy(s.done);
        }
        if (s.host) (void)hipHostFree(s.host);
        if (s.dev) (void)hipFree(s.dev);
    }
    for (auto* v : {&h->prof_used, &h->prof_free})
        for (auto& pe : *v)
            for (auto& e : pe.e) (void)hipEventDestroy(e);
    if (h->step_done) {
        (void)hipEventSynchronize(h->step_done);
        (void)hipEventDestroy(h->step_done);
    }
    if (h->d_queue) (void)hipFree(h->d_queue);
    if (h->obs_host) (void)hipHostFree(h->obs_host);
    if (h->na_done) {
        (void)hipEventSynchronize(h->na_done);
        (void)hipEventDestroy(h->na_done);
    }
    if (h->na_host) (void)hipHostFree(h->na_host);
    if (h->d_tab64) (void)hipFree(h->d_tab64);
    if (h->d_tab32) (void)hipFree(h->d_tab32);
    delete h;
}

static int grid_for(const sfq_ctx* h, size_t n, int per_cu = 8)
{
    const size_t blocks = (n + 255) / 256;
    const size_t cap = (size_t)h->num_cus * per_cu;
    return (int)std::max<size_t>(1, std::min(blocks, cap));
}

extern "C" {

sfq_status sfq_create(const sfq_config* cfg, sfq_handle* out)
{
    if (!cfg || !out) return fail(nullptr, SFQ_E_ARG, "sfq_create: NULL argument");
    *out = nullptr;
    const bool have_w = cfg->ref_omega > 0.0, have_l = cfg->ref_length > 0.0;
    if (have_w == have_l)
        return fail(nullptr, SFQ_E_ARG, "sfq_create: exactly one of ref_omega, ref_length must be > 0");
    if (!(cfg->dt > 0.0) || !std::isfinite(cfg->dt))
        return fail(nullptr, SFQ_E_ARG, "sfq_create: dt must be positive and finite");
    if (cfg->precision != SFQ_FP64 && cfg->precision != SFQ_MIXED)
        return fail(nullptr, SFQ_E_ARG, "sfq_create: bad precision");
    if (cfg->decision != SFQ_OPTICAL_DEPTH && cfg->decision != SFQ_LOCAL)
        return fail(nullptr, SFQ_E_ARG, "sfq_create: bad decision");
    if (cfg->blcfa && cfg->decision != SFQ_LOCAL)
        return fail(nullptr, SFQ_E_ARG, "sfq_create: beyond-LCFA emission requires the local decision");
    if (cfg->approx != SFQ_APPROX_FULL && cfg->approx != SFQ_APPROX_TRUNCATED)
        return fail(nullptr, SFQ_E_ARG, "sfq_create: bad approx");
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0)
        return fail(nullptr, SFQ_E_DEVICE, "sfq_create: no HIP device");
    if (cfg->device < 0 || cfg->device >= ndev)
        return fail(nullptr, SFQ_E_ARG, "sfq_create: device ordinal out of range");
    sfq_ctx* h = new sfq_ctx();
    h->device = cfg->device;
    if (hipSetDevice(h->device) != hipSuccess) {
        delete h;
        return fail(nullptr, SFQ_E_DEVICE, "sfq_create: hipSetDevice failed");
    }
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, h->device) == hipSuccess && prop.multiProcessorCount > 0)
        h->num_cus = prop.multiProcessorCount;
    const double lambda_r = have_l ? cfg->ref_length : C_LIGHT / cfg->ref_omega;
    h->lc_over_lr = LAMBDA_C / lambda_r;
    h->lr_over_lc = lambda_r / LAMBDA_C;
    h->dt = cfg->dt;
    h->precision = cfg->precision;
    h->decision = cfg->decision;
    h->blcfa = cfg->blcfa;
    h->bw_fast = cfg->bw_fast;
    h->ph.dt = cfg->dt;
    h->ph.lc_over_lr = h->lc_over_lr;
    h->ph.k_rate = ALPHA / (sqrt(3.0) * PI) * h->lr_over_lc;
    h->ph.chi_min_pair = cfg->bw_fast ? 0.3 : 0.01;
    const sfq_status st = load_tables(h, cfg->tables_path);
    if (st != SFQ_OK) {
        const std::string msg = tl_error;
        release(h);
        tl_error = msg;
        return st;
    }
    h->approx = cfg->approx;
    h->ph.trunc = h->tb.trunc = (cfg->approx == SFQ_APPROX_TRUNCATED) ? 1 : 0;
    // the emitter kernel's observations for sizing the emitter queue: pinned host memory the
    // kernel writes directly (without it the queue keeps its initial size)
    void* obs = nullptr;
    if (hipHostMalloc(&obs, 256, hipHostMallocMapped) == hipSuccess) {
        void* dptr = nullptr;
        if (hipHostGetDevicePointer(&dptr, obs, 0) == hipSuccess) {
            h->obs_host = (unsigned*)obs;
            h->obs_dev = (unsigned*)dptr;
            memset(obs, 0, 256);
        } else {
            (void)hipHostFree(obs);
        }
    }
    // the step that allocates nothing: the device address of the static scratch (once per
    // device, with the device current), a pinned descriptor buffer and its event
    {
        std::lock_guard<std::mutex> lock(g_scratch_mu);
        if ((int)g_scratch_ptr.size() <= h->device) g_scratch_ptr.resize(h->device + 1, nullptr);
        if (!g_scratch_ptr[h->device]) {
            void* ptr = nullptr;
            if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) == hipSuccess && ptr)
                g_scratch_ptr[h->device] = ptr;
        }
        h->na_scratch = g_scratch_ptr[h->device];
    }
    if (h->na_scratch) {
        if (hipHostMalloc(&h->na_host, STAGING_BYTES, hipHostMallocDefault) != hipSuccess)
            h->na_host = nullptr;
        if (hipEventCreateWithFlags(&h->na_done, hipEventDisableTiming) != hipSuccess)
            h->na_done = nullptr;
    }
    (void)hipGetLastError();
    *out = h;
    return SFQ_OK;
}

void sfq_destroy(sfq_handle h) { release(h); }

const char* sfq_last_error(sfq_handle h)
{
    (void)h;
    return tl_error.c_str();
}

sfq_status sfq_units(sfq_handle h, double* lc_over_lr, double* lr_over_lc)
{
    if (!h) return fail(h, SFQ_E_STATE, "sfq_units: NULL handle");
    if (lc_over_lr) *lc_over_lr = h->lc_over_lr;
    if (lr_over_lc) *lr_over_lc = h->lr_over_lc;
    return SFQ_OK;
}

sfq_status sfq_chi(sfq_handle h, int species, size_t n, const double* px, const double* py,
                   const double* pz, const double* ex, const double* ey, const double* ez,
                   const double* bx, const double* by, const double* bz, double* gamma_out,
                   double* chi_out, void* stream)
{
    if (!h) return fail(h, SFQ_E_STATE, "sfq_chi: NULL handle");
    if (species < 0 || species > 2) return fail(h, SFQ_E_ARG, "sfq_chi: bad species");
    if (n == 0) return SFQ_OK;
    if (!px || !py || !pz || !ex || !ey || !ez || !bx || !by || !bz || !chi_out)
        return fail(h, SFQ_E_ARG, "sfq_chi: NULL array");
    HIP_TRY(h, hipSetDevice(h->device));
    hipLaunchKernelGGL(chi_kernel, dim3(grid_for(h, n)), dim3(256), 0, (hipStream_t)stream,
                       species == SFQ_PHOTON, n, px, py, pz, ex, ey, ez, bx, by, bz,
                       h->lc_over_lr, gamma_out, chi_out);
    HIP_TRY(h, hipGetLastError());
    return SFQ_OK;
}

sfq_status sfq_rates(sfq_handle h, int species, size_t n, const double* gamma, const double* chi,
                     double* rate_out, void* stream)
{
    if (!h) return fail(h, SFQ_E_STATE, "sfq_rates: NULL handle");
    if (species < 0 || species > 2) return fail(h, SFQ_E_ARG, "sfq_rates: bad species");
    if (n == 0) return SFQ_OK;
    if (!gamma || !chi || !rate_out) return fail(h, SFQ_E_ARG, "sfq_rates: NULL array");
    HIP_TRY(h, hipSetDevice(h->device));
    const int photon = species == SFQ_PHOTON;
    if (h->precision == SFQ_MIXED)
        hipLaunchKernelGGL(rates_kernel<true>, dim3(grid_for(h, n)), dim3(256), 0,
                           (hipStream_t)stream, h->tb, h->ph, photon, n, gamma, chi, rate_out);
    else
        hipLaunchKernelGGL(rates_kernel<false>, dim3(grid_for(h, n)), dim3(256), 0,
                           (hipStream_t)stream, h->tb, h->ph, photon, n, gamma, chi, rate_out);
    HIP_TRY(h, hipGetLastError());
    return SFQ_OK;
}

sfq_status sfq_sample_photon(sfq_handle h, size_t n, const double* gamma, const double* chi,
                             const double* r, double* gamma_photon_out, double* gamma_emitter_out,
                             void* stream)
{
    if (!h) return fail(h, SFQ_E_STATE, "sfq_sample_photon: NULL handle");
    if (n == 0) return SFQ_OK;
    if (!gamma || !chi || !r || !gamma_photon_out)
        return fail(h, SFQ_E_ARG, "sfq_sample_photon: NULL array");
    HIP_TRY(h, hipSetDevice(h->device));
    if (h->precision == SFQ_MIXED)
        hipLaunchKernelGGL(sample_photon_kernel<true>, dim3(grid_for(h, n)), dim3(256), 0,
                           (hipStream_t)stream, h->tb, n, gamma, chi, r, gamma_photon_out,
                           gamma_emitter_out);
    else
        hipLaunchKernelGGL(sample_photon_kernel<false>, dim3(grid_for(h, n)), dim3(256), 0,
                           (hipStream_t)stream, h->tb, n, gamma, chi, r, gamma_photon_out,
                           gamma_emitter_out);
    HIP_TRY(h, hipGetLastError());
    return SFQ_OK;
}

sfq_status sfq_sample_pair(sfq_handle h, size_t n, const double* gamma, const double* chi,
                           const double* r, double* gamma_electron_out,
                           double* gamma_positron_out, void* stream)
{
    if (!h) return fail(h, SFQ_E_STATE, "sfq_sample_pair: NULL handle");
    if (n == 0) return SFQ_OK;
    if (!gamma || !chi || !r || !gamma_electron_out)
        return fail(h, SFQ_E_ARG, "sfq_sample_pair: NULL array");
    HIP_TRY(h, hipSetDevice(h->device));
    if (h->precision == SFQ_MIXED)
        hipLaunchKernelGGL(sample_pair_kernel<true>, dim3(grid_for(h, n)), dim3(256), 0,
                           (hipStream_t)stream, h->tb, n, gamma, chi, r, gamma_electron_out,
                           gamma_positron_out);
    else
        hipLaunchKernelGGL(sample_pair_kernel<false>, dim3(grid_for(h, n)), dim3(256), 0,
                           (hipStream_t)stream, h->tb, n, gamma, chi, r, gamma_electron_out,
                           gamma_positron_out);
    HIP_TRY(h, hipGetLastError());
    return SFQ_OK;
}

sfq_status sfq_philox(sfq_handle h, size_t n, const uint64_t* uid, uint64_t seed, uint64_t step,
                      uint32_t purpose, uint64_t* a_out, uint64_t* b_out, void* stream)
{
    if (!h) return fail(h, SFQ_E_STATE, "sfq_philox: NULL handle");
    if (n == 0) return SFQ_OK;
    if (!uid || !a_out) return fail(h, SFQ_E_ARG, "sfq_philox: NULL array");
    HIP_TRY(h, hipSetDevice(h->device));
    hipLaunchKernelGGL(philox_kernel, dim3(grid_for(h, n)), dim3(256), 0, (hipStream_t)stream, n,
                       uid, seed, (uint32_t)step, purpose, a_out, b_out);
    HIP_TRY(h, hipGetLastError());
    return SFQ_OK;
}

sfq_status sfq_init_optical_depth(sfq_handle h, size_t n, const uint64_t* uid, uint64_t seed,
                                  double* tau_out, void* stream)
{
    if (!h) return fail(h, SFQ_E_STATE, "sfq_init_optical_depth: NULL handle");
    if (n == 0) return SFQ_OK;
    if (!uid || !tau_out) return fail(h, SFQ_E_ARG, "sfq_init_optical_depth: NULL array");
    HIP_TRY(h, hipSetDevice(h->device));
    hipLaunchKernelGGL(init_tau_kernel, dim3(grid_for(h, n)), dim3(256), 0, (hipStream_t)stream, n,
                       uid, seed, tau_out);
    HIP_TRY(h, hipGetLastError());
    return SFQ_OK;
}

sfq_status sfq_set_launch(sfq_handle h, int blocks_per_cu, int chunk)
{
    if (!h) return fail(h, SFQ_E_STATE, "sfq_set_launch: NULL handle");
    if (blocks_per_cu < 1 || blocks_per_cu > 64 || chunk < STEP_BLOCK || chunk > (1 << 22) ||
        chunk % STEP_BLOCK != 0)
        return fail(h, SFQ_E_ARG, "sfq_set_launch: blocks_per_cu in [1, 64], chunk a multiple of "
                                  "256 in [256, 2^22]");
    std::lock_guard<std::mutex> lock(h->mu);
    h->blocks_per_cu = blocks_per_cu;
    h->chunk = chunk;
    return SFQ_OK;
}

sfq_status sfq_get_launch(sfq_handle h, int* blocks_per_cu, int* chunk)
{
    if (!h) return fail(h, SFQ_E_STATE, "sfq_get_launch: NULL handle");
    if (blocks_per_cu) *blocks_per_cu = h->blocks_per_cu;
    if (chunk) *chunk = h->chunk;
    return SFQ_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------------------------
// Step plumbing shared by sfq_step and the plans
// ---------------------------------------------------------------------------------------------
static sfq_status validate_desc(sfq_ctx* h, const sfq_step_desc* desc, std::vector<uint32_t>& off,
                                int chunk)
{
    if (!desc || !desc->tiles) return fail(h, SFQ_E_ARG, "sfq_step: NULL descriptor");
    if (desc->ntiles <= 0 || desc->ntiles > SFQ_MAX_TILES)
        return fail(h, SFQ_E_ARG, "sfq_step: ntiles out of range");
    if (!desc->counters) return fail(h, SFQ_E_ARG, "sfq_step: NULL counters");
    if (desc->nsets < 0 || desc->nsets > SFQ_MAX_TILES)
        return fail(h, SFQ_E_ARG, "sfq_step: nsets out of range");
    if (desc->nsets == 0 && !desc->product_counts)
        return fail(h, SFQ_E_ARG, "sfq_step: NULL product counts");
    if (desc->nsets > 0 && !desc->product_sets)
        return fail(h, SFQ_E_ARG, "sfq_step: NULL product sets");
    if (desc->push != 0 && desc->push != 1)
        return fail(h, SFQ_E_ARG, "sfq_step: push must be 0 or 1");
    if (desc->zero_product_counts != 0 && desc->zero_product_counts != 1)
        return fail(h, SFQ_E_ARG, "sfq_step: zero_product_counts must be 0 or 1");
    const int nt = desc->ntiles;
    off.assign(nt + 1, 0);
    for (int t = 0; t < nt; ++t) {
        const sfq_tile& T = desc->tiles[t];
        const std::string tn = " (tile " + std::to_string(t) + ")";
        if (T.species < 0 || T.species > 2)
            return fail(h, SFQ_E_ARG, "sfq_step: bad tile species" + tn);
        if (T.field_mode < SFQ_FIELDS_ARRAYS || T.field_mode > SFQ_FIELDS_PLANE_WAVE)
            return fail(h, SFQ_E_ARG, "sfq_step: bad field_mode" + tn);
        if (desc->nsets == 0 ? T.product_set != 0
                             : (T.product_set < 0 || T.product_set >= desc->nsets))
            return fail(h, SFQ_E_ARG, "sfq_step: product set index out of range" + tn);
        if (T.n >= (1ull << 32))
            return fail(h, SFQ_E_CAPACITY, "sfq_step: tile larger than 2^32 - 1 particles");
        const bool photon = T.species == SFQ_PHOTON;
        const bool bl = h->blcfa && !photon;
        if (T.n > 0) {
            if (!T.px || !T.py || !T.pz || !T.uid)
                return fail(h, SFQ_E_ARG, "sfq_step: NULL momentum/uid" + tn);
            const bool fields = !bl || desc->push;
            if (fields && T.field_mode != SFQ_FIELDS_PLANE_WAVE &&
                (!T.ex || !T.ey || !T.ez || !T.bx || !T.by || !T.bz))
                return fail(h, SFQ_E_ARG, "sfq_step: NULL field array" + tn);
            if (fields && T.field_mode == SFQ_FIELDS_PLANE_WAVE) {
                if (!T.wave_amp || !T.wave_phase)
                    return fail(h, SFQ_E_ARG, "sfq_step: NULL plane-wave array" + tn);
                const double* k = T.wave_k;
                const double* e = T.wave_pol;
                const double kk = k[0] * k[0] + k[1] * k[1] + k[2] * k[2];
                const double ee = e[0] * e[0] + e[1] * e[1] + e[2] * e[2];
                const double ke = k[0] * e[0] + k[1] * e[1] + k[2] * e[2];
                if (!(std::fabs(kk - 1.0) < 1e-12 && std::fabs(ee - 1.0) < 1e-12 &&
                      std::fabs(ke) < 1e-12) || !std::isfinite(T.wave_phase0))
                    return fail(h, SFQ_E_ARG,
                                "sfq_step: plane wave needs unit k and e with k.e = 0" + tn);
            }
            if (!bl && h->decision == SFQ_OPTICAL_DEPTH && !T.tau)
                return fail(h, SFQ_E_ARG, "sfq_step: NULL tau" + tn);
            if (photon && !T.alive)
                return fail(h, SFQ_E_ARG, "sfq_step: photon tiles need an alive array" + tn);
            if (bl && ((!desc->push && (!T.px_prev || !T.py_prev || !T.pz_prev)) || !T.fperp ||
                       !T.dfperp || !T.just_created))
                return fail(h, SFQ_E_ARG, "sfq_step: beyond-LCFA state missing" + tn);
        }
        const uint64_t nch = (T.n + chunk - 1) / chunk;
        if ((uint64_t)off[t] + nch >= (1ull << 29))
            return fail(h, SFQ_E_CAPACITY, "sfq_step: too many particles in one step (at most "
                                           "2^29 - 1 chunks)");
        off[t + 1] = off[t] + (uint32_t)nch;
    }
    auto bad = [](const sfq_products& P) {
        return P.capacity > 0 && (!P.px || !P.py || !P.pz || !P.tau || !P.uid || !P.parent);
    };
    if (desc->nsets == 0) {
        if (bad(desc->photons) || bad(desc->electrons) || bad(desc->positrons))
            return fail(h, SFQ_E_ARG, "sfq_step: NULL product array");
    } else {
        for (int k = 0; k < desc->nsets; ++k) {
            const sfq_product_set& S = desc->product_sets[k];
            if (!S.product_counts || bad(S.photons) || bad(S.electrons) || bad(S.positrons))
                return fail(h, SFQ_E_ARG, "sfq_step: NULL array in product set " + std::to_string(k));
        }
    }
    return SFQ_OK;
}

// The most chunks one streaming block may take: its even share and a sixteenth more (at least
// one), so that fast blocks take over from slow ones at the end of the step (none more below 4
// chunks per block, where a step is short and a larger worst case would only defer shares).
// The queue's worst case is sized for it.  A small surplus keeps the emitter blocks' work,
// which follows the streaming blocks' slices, nearly even.
static int max_chunks_per_block(int nchunks, int grid)
{
    const int even = (nchunks + grid - 1) / grid;
    return even + (even >= 4 ? std::max(1, even / 16) : 0);
}

struct QueueShape {
    int grid;                // streaming blocks
    int max_chunks;          // max_chunks_per_block
    uint64_t slices;         // grid * STEP_WAVES: one per wave
    uint64_t cap_per_wave;   // entries of a slice
    uint64_t entries;        // slices * cap_per_wave
    uint64_t deferrable;     // STEP_WAVES * chunks: the most shares a step can defer
    int may_defer;           // cap_per_wave is below the worst case (every particle emitting)
};

// The queue of a step of nchunks chunks.  A wave's slice holds one share of a chunk (what one
// chunk can add to it) plus the fraction `frac` of every particle of the wave's shares (the
// expected emitters with headroom), at most all of them: then no share is ever deferred.
static QueueShape queue_shape(const sfq_ctx* h, int nchunks, int blocks_per_cu, int chunk,
                              double frac)
{
    QueueShape q;
    q.grid = std::max(1, std::min(nchunks, h->num_cus * blocks_per_cu));
    q.slices = (uint64_t)q.grid * STEP_WAVES;
    q.max_chunks = max_chunks_per_block(nchunks, q.grid);
    const uint64_t chunks_per_block = (uint64_t)q.max_chunks;
    const uint64_t share = (uint64_t)chunk / STEP_WAVES;
    const uint64_t worst = chunks_per_block * share;
    const double want = (double)share + std::ceil(std::max(0.0, frac) * (double)worst);
    q.cap_per_wave = std::max<uint64_t>(1, std::min<uint64_t>(worst, (uint64_t)want));
    q.may_defer = q.cap_per_wave < worst ? 1 : 0;
    q.entries = q.slices * q.cap_per_wave;
    q.deferrable = (uint64_t)STEP_WAVES * (uint64_t)std::max(nchunks, 1);
    return q;
}

// Bytes per queue entry for the handle's form: chi, gamma, p (5 doubles) and index and tile
// (2 uint32), plus the uid with local decisions and the two beyond-LCFA values.
static size_t queue_entry_bytes(const sfq_ctx* h)
{
    return 48 + (h->decision == SFQ_LOCAL ? 8 : 0) + (h->blcfa ? 16 : 0);
}

// Queue memory: the control words (d_ctl, the first 256 bytes), per slice 2 counts, per
// streaming block their 2 sums, its chunk count and its processed count, the deferred-share
// list, then the entries.
struct QueueLayout {
    size_t count, sbcount, proc, dlist, soa, total;
};

static QueueLayout queue_layout(const sfq_ctx* h, const QueueShape& q)
{
    auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
    QueueLayout L;
    L.count = 256;
    L.sbcount = al(L.count + 8 * q.slices);
    L.proc = al(L.sbcount + 16 * (size_t)q.grid);
    L.dlist = al(L.proc + 8 * (size_t)q.grid);
    L.soa = al(L.dlist + 4 * q.deferrable);
    L.total = L.soa + q.entries * queue_entry_bytes(h);
    return L;
}

static size_t queue_bytes(const sfq_ctx* h, const QueueShape& q) { return queue_layout(h, q).total; }

// Emitter blocks per streaming block's slices: enough emitter blocks to keep every compute unit
// busy with the latency-bound emitter pass even when the streaming pass runs few, large blocks;
// twice as many after a step whose emitters were dense, as each block then has several rounds
// of emitters to chain.
#ifndef SFQ_EMIT_BPC
#define SFQ_EMIT_BPC 6
#endif
static int emit_split_for(const sfq_ctx* h, int grid)
{
    const int bpc = h->emit_frac > DENSE_EMITTER_FRACTION ? 2 * SFQ_EMIT_BPC : SFQ_EMIT_BPC;
    return std::max(1, std::min(16, (h->num_cus * bpc) / std::max(1, grid)));
}

// The arrays of a queue allocated with the capacities `cap` at `mem`, bound for a step of shape
// qs (qs fits cap): the fields a form does not use are not allocated, and their pointers are
// null (the kernels touch them only in the forms that use them).
static void bind_queue(const sfq_ctx* h, StepArgs& A, void* mem, const QueueShape& cap,
                       const QueueShape& qs)
{
    const QueueLayout L = queue_layout(h, cap);
    char* base = (char*)mem;
    char* q = base + L.soa;
    const size_t E = cap.entries;
    A.q_chi = (double*)q;
    A.q_gamma = (double*)(q + 8 * E);
    A.q_px = (double*)(q + 16 * E);
    A.q_py = (double*)(q + 24 * E);
    A.q_pz = (double*)(q + 32 * E);
    size_t pos = 40 * E;
    A.q_uid = nullptr;
    A.q_aux = A.q_aux2 = nullptr;
    if (h->decision == SFQ_LOCAL) {
        A.q_uid = (uint64_t*)(q + pos);
        pos += 8 * E;
    }
    if (h->blcfa) {
        A.q_aux = (double*)(q + pos);
        A.q_aux2 = (double*)(q + pos + 8 * E);
        pos += 16 * E;
    }
    A.q_idx = (uint32_t*)(q + pos);
    A.q_tile = (uint32_t*)(q + pos + 4 * E);
    A.d_ctl = (unsigned*)base;
    A.q_count = (uint32_t*)(base + L.count);
    A.q_sbcount = (uint32_t*)(base + L.sbcount);
    A.q_proc = (unsigned long long*)(base + L.proc);
    A.d_list = (uint32_t*)(base + L.dlist);
    A.q_cap_per_wave = qs.cap_per_wave;
    A.grid = qs.grid;
    A.max_chunks = qs.max_chunks;
    A.obs = nullptr;
    A.emit_obs = h->obs_host ? h->obs_dev + 2 : nullptr;
    A.may_defer = qs.may_defer;
}

static bool queue_fits(const QueueShape& cap, const QueueShape& qs)
{
    return qs.entries <= cap.entries && qs.slices <= cap.slices && qs.grid <= cap.grid &&
           qs.deferrable <= cap.deferrable;
}

static void fill_args(const sfq_ctx* h, const sfq_step_desc* desc, StepArgs& A, int nchunks,
                      int chunk)
{
    A.tb = h->tb;
    A.ph = h->ph;
    A.ntiles = desc->ntiles;
    A.nchunks = nchunks;
    A.chunk = chunk;
    A.decision = h->decision;
    A.blcfa = h->blcfa;
    A.step = (uint32_t)desc->step;
    A.step_ptr = nullptr;
    A.seed = desc->seed;
    A.prod[0] = desc->photons;
    A.prod[1] = desc->electrons;
    A.prod[2] = desc->positrons;
    A.prod_counts = desc->product_counts;
    A.counters = desc->counters;
    A.sets = nullptr;
    A.nsets = desc->nsets;
    A.push = desc->push;
    A.zero_counts = desc->zero_product_counts;
    A.wave = 0;
    for (int t = 0; t < desc->ntiles; ++t)
        if (desc->tiles[t].field_mode == SFQ_FIELDS_PLANE_WAVE) A.wave = 1;
}

// A set of timing events for one step (caller holds h->mu); nullptr when timing is off or the
// events cannot be created (timing is instrumentation: it never fails a step).
static ProfEvents* prof_events(sfq_ctx* h)
{
    if (!h->prof) return nullptr;
    if (h->prof_free.empty()) {
        ProfEvents pe{};
        for (auto& e : pe.e)
            // timing only: no system-scope fence on record (a cache writeback and invalidation
            // per event would slow the steps being timed)
            if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess)
                return nullptr;
        h->prof_free.push_back(pe);
    }
    h->prof_used.push_back(h->prof_free.back());
    h->prof_free.pop_back();
    h->prof_used.back().split = h->prof == 1;
    return &h->prof_used.back();
}

// The step's kernels, with the timing events (pe: before the streaming kernel, between it and
// the emitter pass when the timing is split, after the step's last kernel) when the step is
// timed.
static void launch_step_kernels(const sfq_ctx* h, const StepArgs& A, int grid, hipStream_t st,
                                const ProfEvents* pe = nullptr)
{
    const dim3 g(grid), b(STEP_BLOCK);
    if (pe) (void)hipEventRecord(pe->e[0], st);
    const bool mixed = h->precision == SFQ_MIXED, local = h->decision == SFQ_LOCAL;
    const dim3 ge(grid * A.emit_split);
#define SFQ_LAUNCH_FORM(K, G, M, BL, L, X)                                                     \
    do {                                                                                       \
        if (X.push) {                                                                          \
            if (X.wave) hipLaunchKernelGGL((K<M, BL, L, true, true>), G, b, 0, st, X);         \
            else hipLaunchKernelGGL((K<M, BL, L, true, false>), G, b, 0, st, X);               \
        } else {                                                                               \
            if (X.wave) hipLaunchKernelGGL((K<M, BL, L, false, true>), G, b, 0, st, X);        \
            else hipLaunchKernelGGL((K<M, BL, L, false, false>), G, b, 0, st, X);              \
        }                                                                                      \
    } while (0)
#define SFQ_LAUNCH_ARGS(K, G, X)                                                               \
    do {                                                                                       \
        if (h->blcfa) {                                                                        \
            if (mixed) SFQ_LAUNCH_FORM(K, G, true, true, true, X);                             \
            else SFQ_LAUNCH_FORM(K, G, false, true, true, X);                                  \
        } else if (mixed) {                                                                    \
            if (local) SFQ_LAUNCH_FORM(K, G, true, false, true, X);                            \
            else SFQ_LAUNCH_FORM(K, G, true, false, false, X);                                 \
        } else {                                                                               \
            if (local) SFQ_LAUNCH_FORM(K, G, false, false, true, X);                           \
            else SFQ_LAUNCH_FORM(K, G, false, false, false, X);                                \
        }                                                                                      \
    } while (0)
#define SFQ_LAUNCH_EMIT(K, G, X)                                                               \
    do {                                                                                       \
        if (mixed) {                                                                           \
            if (h->blcfa) hipLaunchKernelGGL((K<true, true, true>), G, b, 0, st, X);           \
            else if (local) hipLaunchKernelGGL((K<true, false, true>), G, b, 0, st, X);        \
            else hipLaunchKernelGGL((K<true, false, false>), G, b, 0, st, X);                  \
        } else {                                                                               \
            if (h->blcfa) hipLaunchKernelGGL((K<false, true, true>), G, b, 0, st, X);          \
            else if (local) hipLaunchKernelGGL((K<false, false, true>), G, b, 0, st, X);       \
            else hipLaunchKernelGGL((K<false, false, false>), G, b, 0, st, X);                 \
        }                                                                                      \
    } while (0)
    SFQ_LAUNCH_ARGS(bulk_kernel, g, A);
    if (pe && pe->split) (void)hipEventRecord(pe->e[1], st);
    SFQ_LAUNCH_EMIT(emit_kernel, ge, A);
    // the deferred shares, when the queue may have been too small for some
    const dim3 gd(2 * h->num_cus);
    if (A.may_defer) SFQ_LAUNCH_ARGS(defer_kernel, gd, A);
#undef SFQ_LAUNCH_EMIT
#undef SFQ_LAUNCH_ARGS
#undef SFQ_LAUNCH_FORM
    if (pe) (void)hipEventRecord(pe->e[2], st);
}

struct sfq_plan_t {
    sfq_ctx* h = nullptr;
    StepArgs A{};
    int grid = 0;
    int zero_counts = 0;
    void* d_mem = nullptr;                // descriptors, chunk offsets, step counter, queue
    unsigned long long* d_step = nullptr;
    hipStream_t cap_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int graph_steps = 0;
};

static void plan_release(sfq_plan_t* p)
{
    if (!p) return;
    if (p->h) (void)hipSetDevice(p->h->device);
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    if (p->cap_stream) (void)hipStreamDestroy(p->cap_stream);
    if (p->d_mem) (void)hipFree(p->d_mem);
    delete p;
}

// Zeroes the product counts of a step with product sets (a kernel, not a memset, so graphs
// replay it safely).  Steps without sets need none: their emitter kernel starts from zero.
static void enqueue_zero_counts(const StepArgs& A, hipStream_t st)
{
    if (A.nsets > 0)
        hipLaunchKernelGGL(zero_set_counts_kernel, dim3((3 * A.nsets + 255) / 256), dim3(256), 0, st,
                           A.sets, A.nsets);
}

static void plan_enqueue(sfq_plan_t* p, hipStream_t st, const ProfEvents* pe = nullptr)
{
    if (p->zero_counts) enqueue_zero_counts(p->A, st);
    launch_step_kernels(p->h, p->A, p->grid, st, pe);
    hipLaunchKernelGGL(advance_step_kernel, dim3(1), dim3(64), 0, st, p->d_step);
}

static QueueShape queue_capacity(const sfq_ctx* h)
{
    QueueShape cap;
    cap.may_defer = 0;
    cap.grid = (int)h->q_cap_grid;
    cap.max_chunks = 0;
    cap.slices = h->q_cap_slices;
    cap.entries = h->q_cap_entries;
    cap.deferrable = h->q_cap_deferrable;
    cap.cap_per_wave = 0;
    return cap;
}

// Grows the handle's emitter queue to hold a step of shape qs (caller holds h->mu).  Growing
// waits for the device, since in-flight steps may still use the old queue; a new queue starts
// with its deferral words cleared.
static sfq_status ensure_queue(sfq_ctx* h, const QueueShape& qs, const char* who)
{
    QueueShape cap = queue_capacity(h);
    if (h->d_queue && queue_fits(cap, qs)) return SFQ_OK;
    QueueShape want = qs;
    if (h->d_queue) {
        want.grid = std::max(qs.grid, cap.grid);
        want.slices = std::max(qs.slices, cap.slices);
        want.entries = std::max(qs.entries, cap.entries);
        want.deferrable = std::max(qs.deferrable, cap.deferrable);
        HIP_TRY(h, hipDeviceSynchronize());
        HIP_TRY(h, hipFree(h->d_queue));
        h->d_queue = nullptr;
        h->q_cap_grid = h->q_cap_slices = h->q_cap_entries = h->q_cap_deferrable = 0;
    }
    if (hipMalloc(&h->d_queue, queue_bytes(h, want)) != hipSuccess) {
        h->d_queue = nullptr;
        return fail(h, SFQ_E_NOMEM, std::string(who) + ": cannot allocate the emitter queue");
    }
    HIP_TRY(h, hipMemset(h->d_queue, 0, 256));
    h->q_cap_grid = (uint64_t)want.grid;
    h->q_cap_slices = want.slices;
    h->q_cap_entries = want.entries;
    h->q_cap_deferrable = want.deferrable;
    return SFQ_OK;
}


// What the last completed steps observed (the largest emitter fraction of a wave's share,
// shares deferred): the queue grows to twice the observed fraction, faster after deferrals
// (caller holds h->mu).  The observation may be a step or two old; sizing never changes results.
static void observe_emitters(sfq_ctx* h)
{
    if (!h->obs_host) return;
    volatile unsigned* o = h->obs_host;
    const unsigned fb = o[2];
    if (!fb) return;
    float f;
    memcpy(&f, &fb, sizeof f);
    h->emit_frac = f;
    o[2] = 0;
}

static void adapt_queue(sfq_ctx* h)
{
    observe_emitters(h);
    if (!h->q_adaptive || !h->obs_host) return;
    volatile unsigned* o = h->obs_host;
    const unsigned fb = o[0], nd = o[1];
    if (!(fb | nd)) return;
    float f;
    memcpy(&f, &fb, sizeof f);
    double want = 2.0 * (double)f;
    if (nd) want = std::max(4.0 * (double)f, 2.0 * h->q_frac);
    if (want > h->q_frac) h->q_frac = std::min(1.0, want);
    o[0] = 0;
    o[1] = 0;
}

extern "C" {

sfq_status sfq_reserve(sfq_handle h, uint64_t max_particles, int max_tiles)
{
    if (!h) return fail(h, SFQ_E_STATE, "sfq_reserve: NULL handle");
    if (max_tiles < 1 || max_tiles > SFQ_MAX_TILES)
        return fail(h, SFQ_E_ARG, "sfq_reserve: max_tiles in [1, SFQ_MAX_TILES]");
    std::lock_guard<std::mutex> lock(h->mu);
    const uint64_t nch = (max_particles + h->chunk - 1) / h->chunk + (uint64_t)max_tiles;
    if (nch >= (1ull << 29)) return fail(h, SFQ_E_CAPACITY, "sfq_reserve: too many particles");
    HIP_TRY(h, hipSetDevice(h->device));
    return ensure_queue(h, queue_shape(h, (int)nch, h->blocks_per_cu, h->chunk, h->q_frac),
                        "sfq_reserve");
}

sfq_status sfq_set_queue(sfq_handle h, double expected_fraction, int adaptive)
{
    if (!h) return fail(h, SFQ_E_STATE, "sfq_set_queue: NULL handle");
    if (!(expected_fraction >= 0.0 && expected_fraction <= 1.0) || (adaptive != 0 && adaptive != 1))
        return fail(h, SFQ_E_ARG, "sfq_set_queue: expected_fraction in [0, 1], adaptive 0 or 1");
    std::lock_guard<std::mutex> lock(h->mu);
    h->q_frac = std::min(1.0, 2.0 * expected_fraction);
    h->q_adaptive = adaptive;
    if (h->obs_host) {
        h->obs_host[0] = 0;
        h->obs_host[1] = 0;
    }
    return SFQ_OK;
}

sfq_status sfq_queue_bytes(sfq_handle h, uint64_t* bytes)
{
    if (!h) return fail(h, SFQ_E_STATE, "sfq_queue_bytes: NULL handle");
    if (!bytes) return fail(h, SFQ_E_ARG, "sfq_queue_bytes: NULL output");
    std::lock_guard<std::mutex> lock(h->mu);
    *bytes = h->d_queue ? (uint64_t)queue_bytes(h, queue_capacity(h)) : 0;
    return SFQ_OK;
}

sfq_status sfq_profile_enable(sfq_handle h, int enable)
{
    if (!h) return fail(h, SFQ_E_STATE, "sfq_profile_enable: NULL handle");
    std::lock_guard<std::mutex> lock(h->mu);
    if (enable < 0 || enable > 2)
        return fail(h, SFQ_E_ARG, "sfq_profile_enable: enable must be 0, 1 or 2");
    h->prof = enable;
    return SFQ_OK;
}

sfq_status sfq_profile_read_steps(sfq_handle h, uint64_t max_steps, float* stream_ms,
                                  float* emit_ms, uint64_t* steps)
{
    if (!h) return fail(h, SFQ_E_STATE, "sfq_profile_read_steps: NULL handle");
    std::lock_guard<std::mutex> lock(h->mu);
    if (h->prof_used.size() > max_steps)
        return fail(h, SFQ_E_CAPACITY, "sfq_profile_read_steps: more timed steps than max_steps");
    if (h->prof_used.size() > 0 && (!stream_ms || !emit_ms))
        return fail(h, SFQ_E_ARG, "sfq_profile_read_steps: NULL output arrays");
    HIP_TRY(h, hipSetDevice(h->device));
    uint64_t k = 0;
    for (auto& pe : h->prof_used) {
        HIP_TRY(h, hipEventSynchronize(pe.e[2]));
        if (pe.split) {
            HIP_TRY(h, hipEventElapsedTime(&stream_ms[k], pe.e[0], pe.e[1]));
            HIP_TRY(h, hipEventElapsedTime(&emit_ms[k], pe.e[1], pe.e[2]));
        } else {
            HIP_TRY(h, hipEventElapsedTime(&stream_ms[k], pe.e[0], pe.e[2]));
            emit_ms[k] = 0.0f;
        }
        ++k;
    }
    h->prof_free.insert(h->prof_free.end(), h->prof_used.begin(), h->prof_used.end());
    h->prof_used.clear();
    if (steps) *steps = k;
    return SFQ_OK;
}

sfq_status sfq_profile_read(sfq_handle h, double* stream_ms, double* emit_ms, uint64_t* steps)
{
    if (!h) return fail(h, SFQ_E_STATE, "sfq_profile_read: NULL handle");
    std::lock_guard<std::mutex> lock(h->mu);
    HIP_TRY(h, hipSetDevice(h->device));
    double a = 0, b = 0;
    const uint64_t n = h->prof_used.size();
    for (auto& pe : h->prof_used) {
        HIP_TRY(h, hipEventSynchronize(pe.e[2]));
        float t1 = 0, t2 = 0;
        if (pe.split) {
            HIP_TRY(h, hipEventElapsedTime(&t1, pe.e[0], pe.e[1]));
            HIP_TRY(h, hipEventElapsedTime(&t2, pe.e[1], pe.e[2]));
        } else {
            HIP_TRY(h, hipEventElapsedTime(&t1, pe.e[0], pe.e[2]));
        }
        a += t1;
        b += t2;
    }
    h->prof_free.insert(h->prof_free.end(), h->prof_used.begin(), h->prof_used.end());
    h->prof_used.clear();
    if (stream_ms) *stream_ms = a;
    if (emit_ms) *emit_ms = b;
    if (steps) *steps = n;
    return SFQ_OK;
}

sfq_status sfq_step(sfq_handle h, const sfq_step_desc* desc, void* stream)
{
    if (!h) return fail(h, SFQ_E_STATE, "sfq_step: NULL handle");
    std::lock_guard<std::mutex> lock(h->mu);
    std::vector<uint32_t> off;
    const int chunk = h->chunk;
    const sfq_status v = validate_desc(h, desc, off, chunk);
    if (v != SFQ_OK) return v;
    const int nt = desc->ntiles;
    HIP_TRY(h, hipSetDevice(h->device));
    // A captured step would keep pointers to memory the handle recycles (a staging slot of the
    // descriptors, the emitter queue, which may be reallocated): graphs are made from plans,
    // which own both.
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    HIP_TRY(h, hipStreamIsCapturing((hipStream_t)stream, &cap));
    if (cap != hipStreamCaptureStatusNone)
        return fail(h, SFQ_E_STATE, "sfq_step: the stream is capturing a graph; capture a plan "
                                    "instead (sfq_plan_create, sfq_plan_capture)");
    const int nchunks = (int)off[nt];
    if (nchunks == 0) {
        // nothing to step; the product counts are still zeroed when asked
        if (desc->zero_product_counts) {
            if (desc->nsets > 0) {
                for (int k = 0; k < desc->nsets; ++k)
                    HIP_TRY(h, hipMemsetAsync(desc->product_sets[k].product_counts, 0,
                                              3 * sizeof(unsigned long long),
                                              (hipStream_t)stream));
            } else {
                HIP_TRY(h, hipMemsetAsync(desc->product_counts, 0, 3 * sizeof(unsigned long long),
                                          (hipStream_t)stream));
            }
        }
        return SFQ_OK;
    }
    adapt_queue(h);
    const QueueShape qs = queue_shape(h, nchunks, h->blocks_per_cu, chunk, h->q_frac);
    {
        const sfq_status q = ensure_queue(h, qs, "sfq_step");
        if (q != SFQ_OK) return q;
    }
    // descriptors through a ring of pinned staging buffers and their device copies
    const size_t off_pos = (nt * sizeof(sfq_tile) + 15) & ~(size_t)15;
    const size_t set_pos = (off_pos + (nt + 1) * sizeof(uint32_t) + 15) & ~(size_t)15;
    const size_t used = set_pos + (size_t)desc->nsets * sizeof(sfq_product_set);
    if (used > STAGING_BYTES) return fail(h, SFQ_E_CAPACITY, "sfq_step: too many tiles");
    std::vector<char>& db = h->desc_bytes;
    db.assign(used, 0);
    memcpy(db.data(), desc->tiles, nt * sizeof(sfq_tile));
    memcpy(db.data() + off_pos, off.data(), (nt + 1) * sizeof(uint32_t));
    if (desc->nsets > 0)
        memcpy(db.data() + set_pos, desc->product_sets, desc->nsets * sizeof(sfq_product_set));
    // steps on different streams share the emitter queue: order them on the device
    if (h->any_step && h->last_stream != (hipStream_t)stream)
        HIP_TRY(h, hipStreamWaitEvent((hipStream_t)stream, h->last_end, 0));
    // The same descriptors as the last upload: the kernels read that device copy again, with
    // no copy from the host (a copy costs a transfer and its dispatch latency on every step).
    // Device copies are read-only; a slot is overwritten only after the last step that used it.
    const bool reuse = h->last_slot >= 0 && h->last_desc == db;
    Staging& S = h->staging[reuse ? h->last_slot : h->next_staging];
    if (!reuse) {
        // the slot left behind: every step that read it ends before this point of the stream
        if (h->last_slot >= 0)
            HIP_TRY(h, hipEventRecord(h->staging[h->last_slot].done, (hipStream_t)stream));
        const int slot = h->next_staging;
        h->next_staging = (h->next_staging + 1) % N_STAGING;
        if (!S.host) {
            HIP_TRY(h, hipHostMalloc(&S.host, STAGING_BYTES, hipHostMallocDefault));
            HIP_TRY(h, hipMalloc(&S.dev, STAGING_BYTES));
            HIP_TRY(h, hipEventCreateWithFlags(&S.done, hipEventDisableTiming));
            S.bytes = STAGING_BYTES;
        } else {
            HIP_TRY(h, hipEventSynchronize(S.done));
        }
        memcpy(S.host, db.data(), used);
        HIP_TRY(h, hipMemcpyAsync(S.dev, S.host, used, hipMemcpyHostToDevice,
                                  (hipStream_t)stream));
        h->last_slot = slot;
        h->last_desc.swap(db);
    }
    if (!h->step_done)
        HIP_TRY(h, hipEventCreateWithFlags(&h->step_done, hipEventDisableTiming));
    StepArgs A;
    fill_args(h, desc, A, nchunks, chunk);
    A.tiles = (const sfq_tile*)S.dev;
    A.chunk_off = (const uint32_t*)((char*)S.dev + off_pos);
    if (desc->nsets > 0) A.sets = (const sfq_product_set*)((char*)S.dev + set_pos);
    bind_queue(h, A, h->d_queue, queue_capacity(h), qs);
    A.obs = h->obs_dev;
    A.emit_split = emit_split_for(h, qs.grid);
    if (desc->zero_product_counts) enqueue_zero_counts(A, (hipStream_t)stream);
    const ProfEvents* pe = prof_events(h);
    launch_step_kernels(h, A, qs.grid, (hipStream_t)stream, pe);
    HIP_TRY(h, hipGetLastError());
    // the step's end: its timing event when it is timed (recorded by the launch), else step_done
    // (a timing event recycled after sfq_profile_read and recorded again by a later step then
    // marks a later point of the same handle's ordered steps: waiting for it stays correct)
    if (pe) {
        h->last_end = pe->e[2];
    } else {
        HIP_TRY(h, hipEventRecord(h->step_done, (hipStream_t)stream));
        h->last_end = h->step_done;
    }
    h->last_stream = (hipStream_t)stream;
    h->any_step = true;
    return SFQ_OK;
}

sfq_status sfq_step_noalloc(sfq_handle h, const sfq_step_desc* desc, void* stream)
{
    if (!h) return fail(h, SFQ_E_STATE, "sfq_step_noalloc: NULL handle");
    std::lock_guard<std::mutex> lock(h->mu);
    if (!h->na_scratch || !h->na_host || !h->na_done)
        return fail(h, SFQ_E_STATE, "sfq_step_noalloc: the static scratch of this device could "
                                    "not be set up at sfq_create");
    // the handle's launch shape, with the chunk halved (results never depend on it) until one
    // share per slice takes at most half of the queue's room, so that the rest holds emitters
    const size_t room = NOALLOC_SCRATCH_BYTES - STAGING_BYTES;
    const uint64_t slices = (uint64_t)h->num_cus * (uint64_t)h->blocks_per_cu * STEP_WAVES;
    int chunk = h->chunk;
    while (chunk > STEP_BLOCK &&
           slices * (uint64_t)(chunk / STEP_WAVES) * queue_entry_bytes(h) > room / 2)
        chunk = std::max(STEP_BLOCK, (chunk / 2) & ~(STEP_BLOCK - 1));
    std::vector<uint32_t> off;
    const sfq_status v = validate_desc(h, desc, off, chunk);
    if (v != SFQ_OK) return v;
    const int nt = desc->ntiles;
    HIP_TRY(h, hipSetDevice(h->device));
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    HIP_TRY(h, hipStreamIsCapturing((hipStream_t)stream, &cap));
    if (cap != hipStreamCaptureStatusNone)
        return fail(h, SFQ_E_STATE, "sfq_step_noalloc: the stream is capturing a graph; capture "
                                    "a plan instead (sfq_plan_create, sfq_plan_capture)");
    const int nchunks = (int)off[nt];
    if (nchunks == 0) {
        if (desc->zero_product_counts) {
            if (desc->nsets > 0) {
                for (int k = 0; k < desc->nsets; ++k)
                    HIP_TRY(h, hipMemsetAsync(desc->product_sets[k].product_counts, 0,
                                              3 * sizeof(unsigned long long),
                                              (hipStream_t)stream));
            } else {
                HIP_TRY(h, hipMemsetAsync(desc->product_counts, 0, 3 * sizeof(unsigned long long),
                                          (hipStream_t)stream));
            }
        }
        return SFQ_OK;
    }
    // descriptors: the first STAGING_BYTES of the scratch
    const size_t off_pos = (nt * sizeof(sfq_tile) + 15) & ~(size_t)15;
    const size_t set_pos = (off_pos + (nt + 1) * sizeof(uint32_t) + 15) & ~(size_t)15;
    const size_t used = set_pos + (size_t)desc->nsets * sizeof(sfq_product_set);
    if (used > STAGING_BYTES)
        return fail(h, SFQ_E_CAPACITY, "sfq_step_noalloc: the tile and product-set descriptors "
                                       "exceed the static scratch's " +
                                           std::to_string(STAGING_BYTES) + " bytes for them");
    // the queue: the rest of the scratch, its slices as large as it allows (at most the worst
    // case); shares that do not fit are stepped by the deferred-share kernel
    QueueShape qs = queue_shape(h, nchunks, h->blocks_per_cu, chunk, 1.0);
    const uint64_t worst = qs.cap_per_wave;
    QueueShape probe = qs;
    probe.entries = 0;
    const QueueLayout L0 = queue_layout(h, probe);   // everything but the entries
    const uint64_t per_entry = (uint64_t)queue_entry_bytes(h) * qs.slices;
    if (L0.total + per_entry > room)
        return fail(h, SFQ_E_CAPACITY,
                    "sfq_step_noalloc: " + std::to_string(nchunks) + " chunks of " +
                        std::to_string(chunk) + " particles and " + std::to_string(qs.grid) +
                        " blocks need more than the static scratch of " +
                        std::to_string(NOALLOC_SCRATCH_BYTES) + " bytes (at most about " +
                        std::to_string(room / (4 * STEP_WAVES)) +
                        " chunks; use sfq_step, or a larger chunk)");
    qs.cap_per_wave = std::min<uint64_t>(worst, (room - L0.total) / per_entry);
    qs.entries = qs.slices * qs.cap_per_wave;
    qs.may_defer = qs.cap_per_wave < worst ? 1 : 0;
    // upload: through the handle's pinned buffer, free again once the previous upload is done
    HIP_TRY(h, hipEventSynchronize(h->na_done));
    char* hb = (char*)h->na_host;
    memcpy(hb, desc->tiles, nt * sizeof(sfq_tile));
    memcpy(hb + off_pos, off.data(), (nt + 1) * sizeof(uint32_t));
    if (desc->nsets > 0)
        memcpy(hb + set_pos, desc->product_sets, desc->nsets * sizeof(sfq_product_set));
    char* sc = (char*)h->na_scratch;  // the device address, never the array's name
    HIP_TRY(h, hipMemcpyAsync(sc, hb, used, hipMemcpyHostToDevice, (hipStream_t)stream));
    // the deferral words must start at zero: the deferred-share kernel's last block leaves them
    // so, but the array holds whatever the last call on this device left
    HIP_TRY(h, hipMemsetAsync(sc + STAGING_BYTES, 0, 256, (hipStream_t)stream));
    StepArgs A;
    fill_args(h, desc, A, nchunks, chunk);
    A.tiles = (const sfq_tile*)sc;
    A.chunk_off = (const uint32_t*)(sc + off_pos);
    if (desc->nsets > 0) A.sets = (const sfq_product_set*)(sc + set_pos);
    bind_queue(h, A, sc + STAGING_BYTES, qs, qs);
    observe_emitters(h);
    A.emit_split = emit_split_for(h, qs.grid);
    if (desc->zero_product_counts) enqueue_zero_counts(A, (hipStream_t)stream);
    launch_step_kernels(h, A, qs.grid, (hipStream_t)stream, nullptr);
    HIP_TRY(h, hipGetLastError());
    HIP_TRY(h, hipEventRecord(h->na_done, (hipStream_t)stream));
    return SFQ_OK;
}

sfq_status sfq_plan_create(sfq_handle h, const sfq_step_desc* desc, int zero_product_counts,
                           sfq_plan* out)
{
    if (!h) return fail(h, SFQ_E_STATE, "sfq_plan_create: NULL handle");
    if (!out) return fail(h, SFQ_E_ARG, "sfq_plan_create: NULL output");
    *out = nullptr;
    std::lock_guard<std::mutex> lock(h->mu);
    std::vector<uint32_t> off;
    const int chunk = h->chunk;
    const sfq_status v = validate_desc(h, desc, off, chunk);
    if (v != SFQ_OK) return v;
    const int nt = desc->ntiles;
    const int nchunks = (int)off[nt];
    if (nchunks == 0) return fail(h, SFQ_E_ARG, "sfq_plan_create: no particles");
    HIP_TRY(h, hipSetDevice(h->device));
    const QueueShape qs = queue_shape(h, nchunks, h->blocks_per_cu, chunk, h->q_frac);
    const size_t off_pos = (nt * sizeof(sfq_tile) + 15) & ~(size_t)15;
    const size_t set_pos = (off_pos + (nt + 1) * sizeof(uint32_t) + 15) & ~(size_t)15;
    const size_t step_pos =
        (set_pos + (size_t)desc->nsets * sizeof(sfq_product_set) + 255) & ~(size_t)255;
    const size_t q_pos = step_pos + 256;
    sfq_plan_t* p = new sfq_plan_t();
    p->h = h;
    p->zero_counts = (zero_product_counts || desc->zero_product_counts) ? 1 : 0;
    if (hipMalloc(&p->d_mem, q_pos + queue_bytes(h, qs)) != hipSuccess) {
        p->d_mem = nullptr;
        plan_release(p);
        return fail(h, SFQ_E_NOMEM, "sfq_plan_create: cannot allocate the plan");
    }
    std::vector<char> hostbuf(step_pos + 8, 0);
    memcpy(hostbuf.data(), desc->tiles, nt * sizeof(sfq_tile));
    memcpy(hostbuf.data() + off_pos, off.data(), (nt + 1) * sizeof(uint32_t));
    if (desc->nsets > 0)
        memcpy(hostbuf.data() + set_pos, desc->product_sets, desc->nsets * sizeof(sfq_product_set));
    const unsigned long long step0 = desc->step;
    memcpy(hostbuf.data() + step_pos, &step0, 8);
    if (hipMemcpy(p->d_mem, hostbuf.data(), step_pos + 8, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemset((char*)p->d_mem + q_pos, 0, 256) != hipSuccess ||
        hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking) != hipSuccess) {
        plan_release(p);
        return fail(h, SFQ_E_DEVICE, "sfq_plan_create: device setup failed");
    }
    p->grid = qs.grid;
    p->d_step = (unsigned long long*)((char*)p->d_mem + step_pos);
    fill_args(h, desc, p->A, nchunks, chunk);
    p->A.zero_counts = p->zero_counts;
    p->A.tiles = (const sfq_tile*)p->d_mem;
    p->A.chunk_off = (const uint32_t*)((char*)p->d_mem + off_pos);
    p->A.step_ptr = p->d_step;
    if (desc->nsets > 0) p->A.sets = (const sfq_product_set*)((char*)p->d_mem + set_pos);
    bind_queue(h, p->A, (char*)p->d_mem + q_pos, qs, qs);
    observe_emitters(h);
    p->A.emit_split = emit_split_for(h, qs.grid);
    *out = p;
    return SFQ_OK;
}

void sfq_plan_destroy(sfq_plan p) { plan_release(p); }

sfq_status sfq_plan_launch(sfq_plan p, void* stream)
{
    if (!p) return fail(nullptr, SFQ_E_STATE, "sfq_plan_launch: NULL plan");
    HIP_TRY(p->h, hipSetDevice(p->h->device));
    std::lock_guard<std::mutex> lock(p->h->mu);
    // a launch captured into the caller's graph is not timed
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    HIP_TRY(p->h, hipStreamIsCapturing((hipStream_t)stream, &cap));
    plan_enqueue(p, (hipStream_t)stream,
                 cap == hipStreamCaptureStatusNone ? prof_events(p->h) : nullptr);
    HIP_TRY(p->h, hipGetLastError());
    return SFQ_OK;
}

sfq_status sfq_plan_set_step(sfq_plan p, uint64_t step, void* stream)
{
    if (!p) return fail(nullptr, SFQ_E_STATE, "sfq_plan_set_step: NULL plan");
    HIP_TRY(p->h, hipSetDevice(p->h->device));
    hipLaunchKernelGGL(set_step_kernel, dim3(1), dim3(64), 0, (hipStream_t)stream, p->d_step,
                       (unsigned long long)step);
    HIP_TRY(p->h, hipGetLastError());
    return SFQ_OK;
}

sfq_status sfq_plan_capture(sfq_plan p, int steps)
{
    if (!p) return fail(nullptr, SFQ_E_STATE, "sfq_plan_capture: NULL plan");
    if (steps < 1 || steps > 4096) return fail(p->h, SFQ_E_ARG, "sfq_plan_capture: steps in [1, 4096]");
    HIP_TRY(p->h, hipSetDevice(p->h->device));
    if (p->exec) { HIP_TRY(p->h, hipGraphExecDestroy(p->exec)); p->exec = nullptr; }
    if (p->graph) { HIP_TRY(p->h, hipGraphDestroy(p->graph)); p->graph = nullptr; }
    HIP_TRY(p->h, hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeThreadLocal));
    for (int k = 0; k < steps; ++k) plan_enqueue(p, p->cap_stream);
    hipGraph_t g = nullptr;
    const hipError_t e1 = hipStreamEndCapture(p->cap_stream, &g);
    if (e1 != hipSuccess) return fail(p->h, SFQ_E_DEVICE, std::string("sfq_plan_capture: ") + hipGetErrorString(e1));
    p->graph = g;
    HIP_TRY(p->h, hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0));
    p->graph_steps = steps;
    return SFQ_OK;
}

sfq_status sfq_plan_replay(sfq_plan p, void* stream)
{
    if (!p) return fail(nullptr, SFQ_E_STATE, "sfq_plan_replay: NULL plan");
    if (!p->exec) return fail(p->h, SFQ_E_STATE, "sfq_plan_replay: no graph captured");
    HIP_TRY(p->h, hipSetDevice(p->h->device));
    HIP_TRY(p->h, hipGraphLaunch(p->exec, (hipStream_t)stream));
    return SFQ_OK;
}

}  // extern "C"
