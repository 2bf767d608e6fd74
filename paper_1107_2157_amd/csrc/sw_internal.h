// Internal interface between the C-ABI host code and the HIP kernels of libsw.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

// Device-resident scalars of one solver context.
//  smax[3][64]  ring of max-signal-speed slots, each striped over 64 words
//           (waves spread their atomics over the stripes; a reader takes the
//           max of all 64), as the bit pattern of a non-negative double (so
//           unsigned max == double max).  Step n reads ring slot n%3,
//           max-reduces U^{n+1} into slot (n+1)%3 and clears slot (n+2)%3
//           for step n+1.
constexpr int kStripes = 64;
struct SwScalars {
    unsigned long long smax[3][kStripes];
    double t;                 // simulated time
    double last_dt;           // dt of the last step
    long long steps;          // steps taken
    unsigned int unstable;    // sticky: some step produced h <= 0 or non-finite
    unsigned int pad;
};

// One launch's view of the state and the parameters of the scheme.  Plane
// pointers point at interior cell (0, 0); cell (i, j) is p[j * pitch + i]
// for i in [-1, nx], j in [-1, ny].
struct SwLaunch {
    const void *in[3];
    void *out[3];
    int64_t pitch;
    int32_t nx, ny;
    double g, dx, dy, cfl, dt_fixed;
    int32_t bc_x, bc_y;       // 0 reflect, 1 periodic
    int32_t scheme;           // 0 paper, 1 transverse
    int32_t dtype;            // 0 f32, 1 f64
    SwScalars *sc;
    int32_t step;             // index of this step inside the call (ring position)
    int32_t ghosts;           // 0: the fused step leaves the ghost cells unwritten (TileArgs::ghosts)
};

hipError_t sw_launch_reset(SwScalars *sc, int clear_time, hipStream_t s);
// Fill the halo of `in` (written through in[]) and max-reduce its interior
// signal speed into slot 0.
hipError_t sw_launch_prologue(const SwLaunch &a, hipStream_t s);
hipError_t sw_launch_fill_halo(const SwLaunch &a, hipStream_t s);
// Diagnostics of the interior of `in` (sum h, sum hu, sum hv, max signal
// speed, min h, non-finite cells): the six doubles land at
// scratch[sw_diag_scratch_bytes() / 8 - 6 ...]; scratch holds
// sw_diag_scratch_bytes() bytes of device memory.
size_t sw_diag_scratch_bytes();
hipError_t sw_launch_diagnostics(const SwLaunch &a, double *scratch, hipStream_t s);
// Tuning of a step launch.
struct SwTuning {
    int variant;     // 1 per-cell baseline, 2 fused, 3 temporal blocking (fixed dt; rows = steps per launch),
                     // 4 unfused (face states in HBM), 5 AoS (rows per tile), 6 generated from
                     // region expressions
    int rows;        // fused: rows per tile
    int vec;         // fused: cells per lane
    int minw;        // fused: register budget as waves per SIMD (0 = compiler's choice)
    int pd;          // fused: rows prefetched ahead
    int order;       // fused: tile order (0 XCD row-major, 1 XCD grouped columns of 4, 2 plain)
};
hipError_t sw_launch_step(const SwLaunch &a, const SwTuning &t, hipStream_t s);
hipError_t sw_launch_fused_cfg(const SwLaunch &a, int rows, int vec, int minw, int pd, int order,
                               hipStream_t s);
int sw_fused_default_rows(int nx, int ny, int vec);
// Temporal blocking (fixed dt, paper scheme): k steps of every cell per launch.
bool sw_tb_supported(int dtype, int k);
int sw_tb_tile_rows(int dtype, int k);   // output rows per blocked tile (one grid row of tiles per block row)
// waves per block: 4, 8, 12 or 16 (the tile is the same; each wave marches one chunk of its rows).
hipError_t sw_launch_tb(const SwLaunch &a, int k, int waves, hipStream_t s);
int sw_fused_default_vec(int dtype, int nx);
bool sw_fused_supported(int dtype, int scheme, int vec, int minw, int pd);
// A fused tile of `rows` rows (plus its two halo rows) of `pitch`-element rows
// fits the kernel's 32-bit buffer offsets.
bool sw_fused_tile_fits(int rows, int64_t pitch, int elem_bytes);

// The paper's comparison designs (paper scheme only).  Unfused: face states
// of the first half-step in HBM planes, x face i of row j at x[k][j * pitch
// + i] (i = 0..nx), y face j of column i at y[k][j * pitch + i] (j = 0..ny);
// each plane holds (ny + 1) * pitch elements.
struct SwFaces {
    void *x[3];
    void *y[3];
    int64_t pitch;
};
hipError_t sw_launch_unfused(const SwLaunch &a, const SwFaces &f, hipStream_t s);
// AoS: `rows` rows of `row` elements (halo and padding included) converted
// between the three SoA planes (row stride soa_pitch) and one array of
// (h, hu, hv, 0) vectors (row stride aos_pitch); the step reads and writes
// such arrays (`in`, `out` point at interior cell (0, 0); a.pitch is the AoS
// row stride).
hipError_t sw_launch_aos_convert(int dtype, const void *const soa[3], int64_t soa_pitch, void *aos, int64_t aos_pitch,
                                 int64_t rows, bool to_aos, hipStream_t s);
hipError_t sw_launch_aos_step(const SwLaunch &a, const void *in, void *out, int rows, hipStream_t s);
// The step generated from region expressions (wave_advance.rgn): new
// interior of `out` and the CFL epilogue; the halo is filled separately.
// design 1: LDS tiles of `rows` x 64 (one thread per cell); design 2: a
// row march, `rows` rows per wave (registers and lane shifts, no LDS) with
// `prefetch` input rows loaded ahead of the row being updated (1-3; design 1: 0).
bool sw_rgn_rows_supported(int design, int rows);
hipError_t sw_launch_rgn(const SwLaunch &a, int design, int rows, int prefetch, hipStream_t s);

// The instantiated launch shapes: (dtype, cells per lane, register budget,
// prefetch depth).
#define SW_FUSED_SHAPES(X)                                                                      \
    X(float, 1, 0, 1) X(float, 1, 0, 2) X(float, 1, 4, 2)                                        \
    X(float, 2, 0, 1) X(float, 2, 0, 2) X(float, 2, 0, 3) X(float, 2, 3, 1) X(float, 2, 3, 2)  \
    X(float, 2, 3, 3) X(float, 2, 4, 1) X(float, 2, 4, 2) X(float, 2, 4, 3) X(float, 4, 0, 1)  \
    X(float, 4, 0, 2) X(float, 4, 0, 3) X(float, 4, 3, 1) X(float, 4, 3, 2)                      \
    X(double, 1, 0, 1) X(double, 1, 0, 2) X(double, 1, 0, 3) X(double, 1, 3, 1)                 \
    X(double, 1, 3, 2) X(double, 1, 3, 3) X(double, 1, 4, 1) X(double, 1, 4, 2)                 \
    X(double, 1, 4, 3) X(double, 2, 0, 1) X(double, 2, 0, 2) X(double, 2, 0, 3)                 \
    X(double, 2, 3, 1) X(double, 2, 3, 2)
// The instantiated launch shapes of the transverse scheme (fused and batched
// kernels): default register budget, prefetch depth 1 or 2.
#define SW_FUSED_TR_SHAPES(X)                                                                   \
    X(float, 1, 0, 1) X(float, 1, 0, 2) X(float, 2, 0, 1) X(float, 2, 0, 2) X(float, 4, 0, 1)   \
    X(float, 4, 0, 2) X(double, 1, 0, 1) X(double, 1, 0, 2) X(double, 2, 0, 1) X(double, 2, 0, 2)
