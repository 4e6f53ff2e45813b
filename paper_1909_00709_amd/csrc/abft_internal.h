// Internal declarations shared by the host runtime (abft_runtime.cpp) and the gfx950 kernels
// (abft_kernels.hip).  Not part of the public interface.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <atomic>

#include "abft_stencil.h"

namespace abft {

constexpr int kMaxFlags = 1024;   // flagged rows remembered per sweep for location
constexpr int kMaxMemFlags = 64;  // mismatched input rows remembered per sweep for repair
constexpr int kMaxRecompute = 65536;  // intersection points evaluated again per layer
constexpr int kBatchWaves = 4;  // wavefronts per block of the batched sweep
constexpr int kWideBlockLaneBytes = 64;  // most row bytes per lane for 8-wavefront sweep blocks
constexpr int kFixBlock = 512;    // threads of the single locate/correct block
constexpr int kCheckBlock = 1024; // threads per block of the offline window check
constexpr int kMaxPeriod = 128;   // longest offline window (sweeps per check)
constexpr int kCheckCells = 4;    // checksum-plane cells per thread in the window check
constexpr int kCheckChunk = 16;   // interpolation steps per window-check launch at most
constexpr unsigned kBarrierSpinLimit = 1u << 26;  // polls (~50 ns each) before a grid barrier gives up

// Weight slots of the star stencils of radius 1 and 2: centre, the six face neighbours at
// distance 1 (x-1, x+1, y-1, y+1, z-1, z+1), then the six at distance 2.
enum {
    W_C = 0, W_XM, W_XP, W_YM, W_YP, W_ZM, W_ZP,
    W_XM2, W_XP2, W_YM2, W_YP2, W_ZM2, W_ZP2, W_COUNT
};

// Slot of the tap at distance d (1 or 2) along axis (0 = x, 1 = y, 2 = z), on the minus
// (sign < 0) or plus side.
__host__ __device__ constexpr int w_slot(int axis, int d, int sign)
{
    return (d == 1 ? W_XM : W_XM2) + 2 * axis + (sign > 0 ? 1 : 0);
}

// Slot of tap (dx, dy, dz), each in -1..1, of a 27-point box stencil.
__host__ __device__ constexpr int box_slot(int dx, int dy, int dz)
{
    return (dz + 1) * 9 + (dy + 1) * 3 + (dx + 1);
}

// Dynamic LDS above 64 KiB has to be allowed for each kernel on each device before it is
// launched with it.  One LdsAllowed per kernel instantiation (a function-local static) records
// the largest size allowed so far on each device, so the attribute is set once per size.
constexpr int kMaxDevices = 64;
struct LdsAllowed {
    std::atomic<int> bytes[kMaxDevices];
};
inline hipError_t allow_lds(const void* kern, size_t lds, LdsAllowed& seen)
{
    if (lds <= 65536) return hipSuccess;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    const bool known = dev >= 0 && dev < kMaxDevices;
    if (known && (int)lds <= seen.bytes[dev].load(std::memory_order_relaxed)) return hipSuccess;
    e = hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e == hipSuccess && known) seen.bytes[dev].store((int)lds, std::memory_order_relaxed);
    return e;
}

struct Stencil {
    double w[W_COUNT];  // star weights rounded to the grid dtype, held as double
    uint32_t mask;      // bit k set when slot k is a tap of the stencil
    int32_t bc;         // abft_bc
    double g;           // constant ghost value (rounded to the grid dtype)
    int32_t rad;        // 1, or 2 when a distance-2 tap is present
    int32_t box;        // 1: a 27-point box stencil (taps off the axes); weights in wb
    double wb[27];      // box weights by box_slot (box stencils only)
    uint32_t bmask;     // bit box_slot set for each box tap
    int32_t xterms;     // 1: the x-boundary terms of Theorem 1 do not cancel in the weighted
                        // sum of a row's prediction, so the protected sweep forms them; 0:
                        // they cancel exactly (periodic rule, or clamp with equal x weights)
};

struct RowFlag {
    int32_t z, y;
    int32_t k;              // tile index along x (tile-local checksums), 0 for whole rows
    int32_t pad;
    double direct, pred;
};

// An input row whose sum as the sweep read it differs from the checksum stored with it.
struct MemFlag {
    int32_t z, y;
};

// Both counts are cleared together by the sweep before the one that fills the slot.
struct FlagSlot {
    uint32_t count;               // rows flagged by the output check
    uint32_t mcount;              // input rows flagged by the input check
    RowFlag rows[kMaxFlags];
    MemFlag mrows[kMaxMemFlags];
};

// Device counters; 64-bit so they can be updated with atomicAdd.
struct Counters {
    unsigned long long rows_flagged, cols_flagged, corrected, checksum_faults, uncorrectable;
    unsigned long long windows_checked, windows_flagged, rollbacks, persistent;
    unsigned long long events_total;
    unsigned long long noise_bits;  // bit pattern of the largest non-negative noise (double)
    unsigned long long overflow;    // sweeps whose flagged rows exceeded kMaxFlags
    unsigned long long barrier_timeouts;  // recovery grid barriers that gave up waiting
    unsigned long long mem_flagged, mem_corrected, mem_unlocated;  // input-side check
};

// Sweep kernel variants.
// PROT: checksum, prediction and comparison fused in the sweep; PROTM: PROT plus the check of
// the input rows against their stored checksums and the output's index-weighted row sums.
// TILE: tile-local output sums and tile boundary terms (the check is a separate launch).
enum { MODE_PLAIN = 0, MODE_CSUM = 1, MODE_PROT = 2, MODE_PROTM = 3, MODE_TILE = 4 };
enum { CS_F64 = 0, CS_F32C = 1 };

struct SweepArgs {
    const void* uin;
    void* uout;
    const void* C;          // constant term or null
    double c_scalar;        // constant term when C is null
    Stencil st;
    int32_t nx, ny, nz;
    int32_t tz;             // planes per block
    int32_t nyb, ntiles;    // y-blocks and total tiles (= grid size)
    int32_t attempt;        // fault-plan attempt matched by this sweep
    const int64_t* t_base;  // device sweep base (graph replays) or null
    int64_t t_off;          // sweep index = t_off + (*t_base or 0)
    // checksums
    const double* Bt;       // row checksums of uin (prediction input)
    double* Bn;             // row checksums of uout (written)
    double* Wn;             // index-weighted row sums of uout (written by the PROTM sweep)
    double* Et;             // TILE: boundary terms of the input's tiles (written)
    const double* cB;       // constant-term row checksums
    double eps;
    FlagSlot* slot;         // flagged rows of this sweep
    uint32_t* zero_ptr;     // words cleared by block 0 (next sweep's slot / window counts)
    int32_t zero_n;
    Counters* cnt;
    abft_event* ev;
    int32_t ev_cap;
    int32_t grid;           // grid index reported in events
    // fault plan: entries of sweep t are faults[first[t] .. first[t+1])
    const abft_fault* faults;
    const int32_t* fault_first;
    int64_t fault_tmax;     // first[] covers sweeps [0, fault_tmax)
    // offline
    double* E;              // boundary terms of this sweep's input rows, or null
    const uint32_t* guard;  // run only when *guard != 0 (rollback recompute), or null
};

struct FixArgs {
    const void* uin;        // written only by the repair of input points
    void* uout;
    double* Bn;
    const double* cA;
    // input-side repair (null Wt: none): the input's checksums and weighted sums, the output's
    // weighted sums, and what evaluating an output point again needs
    const double* Bt;
    const double* Wt;
    double* Wn;
    const double* cB;
    const void* C;
    double c_scalar;
    int32_t recompute;      // correct located points by evaluating them again (else Eq.(10))
    int32_t tile_x;         // tile-local checksums of this many points, or 0 (whole rows)
    Stencil st;
    int32_t nx, ny, nz;
    double eps;
    FlagSlot* slot;
    Counters* cnt;
    abft_event* ev;
    int32_t ev_cap;
    int32_t grid;
    const int64_t* t_base;
    int64_t t_off;
};

struct CheckArgs {
    const double* Bin;      // checksums the launch starts from (the checkpoint's, or a chunk's)
    double* Bout;           // interpolated checksums after this launch's steps, or null in the
                            // window's last launch, which compares instead
    const double* Bdir;     // direct checksums at the window end
    const double* cB;
    const double* E;        // [k][nz][ny] boundary terms, or null
    Stencil st;
    int32_t nx, ny, nz;
    int32_t s0, ns;         // the window's steps s0 .. s0 + ns - 1 are done by this launch
    double eps;
    int32_t tyi, tzi, nyt, nzt;   // interior tile sizes and tile counts
    int32_t ry_max, rz_max;       // region extents the LDS was sized for
    uint32_t* flag_count;   // window flag counter written
    const uint32_t* guard;  // run only when *guard != 0, or null
    uint32_t* ticket;       // block-completion counter (reset by the last block)
    Counters* cnt;
    abft_event* ev;
    int32_t ev_cap;
    int32_t attempt;
    int32_t auto_correct;
    int64_t t_first;        // first sweep of the window
    int64_t t_last;         // last sweep of the window
};

// The rollback recompute of an offline window in one launch: the window's k sweeps from the
// checkpoint (attempt 1), separated by grid barriers.
struct RecoverArgs {
    SweepArgs a;                      // fields shared by the window's sweeps
    const void* ckpt;                 // the checkpoint: sweep 0 reads it
    const void* odd;                  // sweep j writes `odd` for even j, `even` for odd j,
    const void* even;                 // and reads what sweep j - 1 wrote
    double* E;                        // [k][nz][ny] boundary terms of the sweeps, or null
    int32_t k;                        // sweeps in the window
    int64_t t_first;                  // first sweep of the window
    const uint32_t* guard;            // run only when *guard != 0, or null
    uint32_t* bar;                    // [0] barrier arrivals, [1] departures; zero between launches
};

// One grid of a batch, as the batched kernels see it.
struct GridDesc {
    void* u[2];             // the grid's two buffers; u[t & 1] holds u^t
    const void* C;
    double c_scalar;
    Stencil st;
    int32_t nx, ny, nz;
    int32_t tz, nyb, ntiles;
    double* B[2];           // B[t & 1] holds the row checksums of u^t
    double* W[2];           // index-weighted row sums beside B (input-side check), or null
    const double* cB;
    const double* cA;
    FlagSlot* slot[2];      // flagged rows of sweeps with t & 1 == index
    int32_t sub;            // chunk count of this grid's rows in its launch: 0 the launch's
                            // nch, 1 its nchb, 2 its nchc
};

struct BatchArgs {
    const GridDesc* grids;
    int32_t ngrids;
    int32_t ntiles;         // tiles of this launch (one size class of grids, or all)
    const int2* order;      // (grid, tile) in processing order (largest first)
    uint32_t* queue;        // persistent launch: [0] next tile, [1] blocks finished
    int32_t persistent;     // 1: blocks pop tiles from the queue; 0: one tile per block
    int32_t zero_slots;     // 1: block 0 clears every grid's next-sweep flag slot (the first
                            // of a sweep's launches)
    int32_t parity;         // t & 1 of this sweep
    const int64_t* t_base;
    int64_t t_off;
    int32_t attempt;
    int32_t recompute;      // locate/correct: evaluate located points again (else Eq.(10))
    double eps;
    Counters* cnt;
    abft_event* ev;
    int32_t ev_cap;
    const abft_fault* faults;
    const int32_t* fault_first;
    int64_t fault_tmax;
};

// Kernel launchers (abft_kernels.hip).  Each returns hipSuccess or the launch error.
struct SweepShape {
    int32_t lpr;   // lanes per row: 16 or 64
    int32_t nch;   // chunks of lpr*vec elements per row: 1, 2, 4 or 8
    int32_t vec;   // elements per 16-byte access (1 for rows that are not 16-byte multiples)
    int32_t tz;    // planes per block
    int32_t pf;    // planes loaded ahead of the one computed: 1 or 2
    int32_t nw = 4;  // wavefronts per block: 4 or 8 (each holds 64 / lpr rows)
    int32_t rad = 1; // stencil radius the kernel is built for: 1 or 2
    int32_t box = 0; // 1: the 27-point box kernel (radius 1, prefetch depth 1)
    // batched radius-1 sweeps: narrower chunk counts one launch also holds (the rows of the
    // grids whose descriptor has sub 1 or 2), 0 for none
    int32_t nchb = 0;
    int32_t nchc = 0;
};

bool sweep_shape_supported(int dtype, const SweepShape& s);
// Dynamic LDS of a sweep block: plane buffers and the per-tile tables (two more tables for
// the input-side check).
size_t sweep_lds_bytes(int dtype, int nx, const SweepShape& s, bool input_check = false);
int sweep_rows_per_block(const SweepShape& s);
hipError_t launch_sweep(int dtype, int mode, int csum, const SweepShape& s, const SweepArgs& a,
                        hipStream_t st);
hipError_t launch_fixup(int dtype, const FixArgs& a, hipStream_t st);
hipError_t launch_fixup_batch(int dtype, const BatchArgs& b, int maxnx, int rad, int box,
                              hipStream_t st);
// Batched sweep (abft_batch.hip): one launch sweeps every grid of the batch.
bool batch_shape_supported(int dtype, const SweepShape& s);
hipError_t launch_sweep_batch(int dtype, int mode, int csum, const SweepShape& s,
                              const BatchArgs& b, int nblocks, size_t lds, hipStream_t st);
size_t batch_lds_bytes(int dtype, int maxnx, int maxtz, const SweepShape& s, bool input_check);
// Batched sweeps of radius-2 stars and 27-point boxes (their own translation units).
// Per stencil form and dtype (batch_{r1,r2,box}_{f32,f64}.hip).
#define ABFT_BATCH_DECL(NAME)                                                                  \
    hipError_t launch_batch_##NAME(int mode, int csum, const SweepShape& s, const BatchArgs& b, \
                                   int nblocks, size_t lds, hipStream_t st);                   \
    int batch_occupancy_##NAME(int mode, int csum, const SweepShape& s, size_t lds);
ABFT_BATCH_DECL(r1_f32)
ABFT_BATCH_DECL(r1_f64)
ABFT_BATCH_DECL(r2_f32)
ABFT_BATCH_DECL(r2_f64)
ABFT_BATCH_DECL(box_f32)
ABFT_BATCH_DECL(box_f64)
ABFT_BATCH_DECL(r1x_f32)  // radius-1 launches holding two or three chunk counts
ABFT_BATCH_DECL(r1x_f64)
#undef ABFT_BATCH_DECL
// Offline, before a rollback recompute (guarded by the window's flag count): the checkpoint's
// rows against their stored checksums, a changed point placed and restored in place.
hipError_t launch_verify_ckpt(int dtype, void* u, const double* Bck, const double* Wck, int nx,
                              int ny, int nz, double eps, const uint32_t* guard, Counters* cnt,
                              abft_event* ev, int cap, int64_t t_first, hipStream_t st);
// Memory-resident faults of the plan for one batched sweep, each in its grid's input buffer.
hipError_t launch_mem_flip_batch(int dtype, const GridDesc* grids, int parity,
                                 const abft_fault* faults, const int32_t* fault_first,
                                 int64_t fault_tmax, const int64_t* t_base, int64_t t_off,
                                 hipStream_t st);
int batch_blocks_per_cu(int dtype, int mode, int csum, const SweepShape& s, size_t lds);
size_t fixup_lds_bytes(int nx, bool box);
hipError_t launch_check(const CheckArgs& a, hipStream_t st);
size_t check_lds_bytes(int ry, int rz);
hipError_t launch_row_sums(int dtype, const void* u, double cs, int nx, int64_t nrows,
                           double* out, hipStream_t st);
// Tile-local checksums: the prediction of every tile's sum (Theorem 1 on the tile) and the
// comparison, after a MODE_TILE sweep.
struct TileCheckArgs {
    const double* Bt;       // tile sums of the input
    const double* Bn;       // tile sums of the output (direct)
    const double* cB;       // tile sums of the constant term
    const double* Et;       // boundary terms of the input's tiles
    Stencil st;
    int32_t nx, ny, nz, tile_x;
    double eps;
    FlagSlot* slot;
    Counters* cnt;
    abft_event* ev;
    int32_t ev_cap;
    int32_t grid;
    const int64_t* t_base;
    int64_t t_off;
};
hipError_t launch_tile_check(const TileCheckArgs& a, hipStream_t st);
hipError_t launch_weighted_row_sums(int dtype, const void* u, int nx, int64_t nrows, double* out,
                                    hipStream_t st);
// Memory-resident faults of the plan for sweep t (kind MEMORY, first attempt): flip them in
// the sweep's input grid u before the sweep reads it.
hipError_t launch_mem_flip(int dtype, void* u, int nx, int ny, const abft_fault* faults,
                           const int32_t* fault_first, int64_t fault_tmax, const int64_t* t_base,
                           int64_t t_off, hipStream_t st);
hipError_t launch_col_sums(int dtype, const void* u, double cs, int nx, int ny, int nz,
                           double* out, hipStream_t st);
hipError_t launch_fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t st);
hipError_t launch_rollback_note(const uint32_t* guard, Counters* cnt, abft_event* ev, int cap,
                                int64_t t_first, int k, hipStream_t st);
// Offline rollback recompute (abft_recover.h), one launch of at most one wave of blocks with
// grid barriers; the shape's lanes, chunks, vector width and wavefronts (prefetch depth 1).
bool recover_shape_supported(int dtype, const SweepShape& s);
hipError_t launch_recover(int dtype, int csum, const SweepShape& s, const RecoverArgs& r,
                          int num_cus, hipStream_t st);
hipError_t launch_recover_f32(int csum, const SweepShape& s, const RecoverArgs& r, size_t lds,
                              int num_cus, hipStream_t st);
hipError_t launch_recover_f64(int csum, const SweepShape& s, const RecoverArgs& r, size_t lds,
                              int num_cus, hipStream_t st);
hipError_t launch_recover_r2_f32(int csum, const SweepShape& s, const RecoverArgs& r, size_t lds,
                                 int num_cus, hipStream_t st);
hipError_t launch_recover_r2_f64(int csum, const SweepShape& s, const RecoverArgs& r, size_t lds,
                                 int num_cus, hipStream_t st);
hipError_t launch_recover_box_f32(int csum, const SweepShape& s, const RecoverArgs& r,
                                  size_t lds, int num_cus, hipStream_t st);
hipError_t launch_recover_box_f64(int csum, const SweepShape& s, const RecoverArgs& r,
                                  size_t lds, int num_cus, hipStream_t st);

// Box (27-point) sweep launchers (prefetch depth 1).
hipError_t launch_sweep_box_f32(int mode, int csum, const SweepShape& s, const SweepArgs& a,
                                hipStream_t st, size_t lds);
hipError_t launch_sweep_box_f64(int mode, int csum, const SweepShape& s, const SweepArgs& a,
                                hipStream_t st, size_t lds);

// Radius-2 sweep launchers (prefetch depth 1).
hipError_t launch_sweep_r2_f32_pc(int mode, int csum, const SweepShape& s, const SweepArgs& a,
                                  hipStream_t st, size_t lds);
hipError_t launch_sweep_r2_f32_prot(int csum, const SweepShape& s, const SweepArgs& a,
                                    hipStream_t st, size_t lds);
hipError_t launch_sweep_r2_f64(int mode, int csum, const SweepShape& s, const SweepArgs& a,
                               hipStream_t st, size_t lds);

// Per-variant sweep launchers (one translation unit each).
#define ABFT_DECL_SWEEP(NAME)                                                                 \
    hipError_t NAME(int csum, const SweepShape& s, const SweepArgs& a, hipStream_t st,         \
                    size_t lds);
ABFT_DECL_SWEEP(launch_sweep_f32_plain)
ABFT_DECL_SWEEP(launch_sweep_f32_csum)
ABFT_DECL_SWEEP(launch_sweep_f32_prot)
ABFT_DECL_SWEEP(launch_sweep_f64_plain)
ABFT_DECL_SWEEP(launch_sweep_f64_csum)
ABFT_DECL_SWEEP(launch_sweep_f64_prot)
ABFT_DECL_SWEEP(launch_sweep_f32_protm)
ABFT_DECL_SWEEP(launch_sweep_f64_protm)
ABFT_DECL_SWEEP(launch_sweep_r2_f32_protm)
ABFT_DECL_SWEEP(launch_sweep_r2_f64_protm)
ABFT_DECL_SWEEP(launch_sweep_box_f32_protm)
ABFT_DECL_SWEEP(launch_sweep_box_f64_protm)
ABFT_DECL_SWEEP(launch_sweep_f32_tile)
ABFT_DECL_SWEEP(launch_sweep_f64_tile)
#undef ABFT_DECL_SWEEP
hipError_t launch_set_i64(int64_t* p, int64_t v, hipStream_t st);

// The allocation-free run (abft_noalloc.hip).  Byte offsets of the workspace of an online or
// plain run inside one device buffer, each 256-byte aligned.
struct NoAllocLayout {
    size_t B[2], W[2], cB, cA, slot[2], cnt, ev, faults, first, total;
    bool wsums;        // index-weighted row sums kept (online with the input check)
    int ev_cap;        // event log capacity
    int64_t tmax;      // one past the fault plan's last sweep
};
// Validates the arguments (no HIP call) and lays the workspace out; ABFT_E_UNSUPPORTED when
// it needs more than `limit` bytes.
abft_status noalloc_layout(const abft_problem* p, const abft_options* o, const abft_fault* f,
                           int32_t nf, size_t limit, NoAllocLayout* L);
// init + inject + step(nsweeps) + check on workspace ws laid out by L, with no allocation.
abft_status run_in_workspace(const abft_problem* p, const abft_options* o, const abft_fault* f,
                             int32_t nf, int64_t nsweeps, void* hip_stream, unsigned char* ws,
                             const NoAllocLayout& L, abft_report* out);
// Records the text of a failed allocation-free run for abft_last_error(NULL); returns s.
abft_status run_error(abft_status s, const char* msg) noexcept;
// first[t] = index of the first fault of a sweep-sorted plan with sweep >= t, t = 0 .. tmax.
hipError_t launch_fault_index(const abft_fault* faults, int32_t n, int32_t* first, int64_t tmax,
                              hipStream_t st);

}  // namespace abft
