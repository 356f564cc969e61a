// Host-side internals shared by the C ABI translation units.
#pragma once
#include <hip/hip_runtime.h>

#include <array>
#include <string>
#include <tuple>
#include <vector>

#include "mhd.h"
#include "mhd_device.h"

namespace mhd {

struct Shape {
    int tx, ty, tz, cz;
    bool pipe;   // true: direct-to-LDS ring kernel (k_pipe); false: register-staged kernel (k_substep)
    bool march;  // true: z-marching column kernel (k_march); tz is its slab depth
    bool zm;     // true: z-marching kernel with register queues (k_zm); a tx x ty column tile
    bool wide;   // zm, FP32: substeps 1 and 2 take 64 x 8 tiles of 1024 threads (substep 0 and
                 // the diagnostics keep the tx x ty tiles and their partials)
};
constexpr int NSHAPES = 16;
constexpr int SHAPE_ZM = 14;
constexpr int SHAPE_ZMW = 15;
constexpr int ZM_WIDE_TX = 64;
extern const Shape SHAPES[NSHAPES];

// steps whose forcing blocks and diagnostic records are staged at once
constexpr int CHUNK = 512;

inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Bytes from one field array to the next in a context's state block.  Fields of at
// least 4 MiB are spaced by their size plus 132.25 KiB: at the plain size (a power of
// two on 2^n grids) the reads of one cell from the fourteen arrays fall at addresses
// that differ only in high bits, and the substeps of a 512^3 FP64 run measured 5-6 %
// slower.  The pad matters beyond that (512^3, z-marching kernel): 132.25 and 196.25
// KiB were the fastest (FP32 substep 2 3 % faster than with 260.25), 68.25 cost FP64
// 1 %, 396.5 and 516.25 cost FP64 4-6 %.
inline size_t field_spacing(size_t ncell, int precision)
{
    const size_t fb = align_up(ncell * (size_t)precision, 256);
    return fb >= ((size_t)4 << 20) ? fb + (128 + 4) * 1024 + 256 : fb;
}

mhd_status fail(mhd_status s, const std::string &msg);
extern thread_local std::string g_err;

}  // namespace mhd

struct mhd_ctx {
    mhd_params p{};
    size_t ncell = 0;
    hipStream_t stream = nullptr;
    int shape = 0;
    bool fit = false;        // halo box spans at most one period per axis (cheap wrap)
    int xs = 0;              // x offset of the tile grid (ring kernel)
    int seg = 0;             // z-segment length of the marching kernel
    int ntiles = 0;
    int ntiles_w = 0;        // 64-wide tiles of substeps 1 and 2 (wide shapes), else 0
    int fstride = 0;
    bool owns = false;
    bool in_batch = false;
    void *mem = nullptr;
    void *bufs[2][mhd::NF] = {};
    int parity = 0;          // buffer set holding the current state
    int64_t step = 0;        // global step index of the current state
    // forcing: 0 none, 1 explicit schedule, 2 random on demand
    int fmode = 0;
    std::vector<mhd_forcing> sched;
    int64_t sched_start = 0;
    double kf = 0, f0 = 0, sigma = 0;
    uint64_t fseed = 0;
    // device scratch: forcing blocks, records, partials, descriptor, tile table
    void *aux = nullptr;
    size_t aux_bytes = 0;
    void *d_forcing = nullptr;
    double *d_records = nullptr;
    double *d_partials = nullptr;
    double *d_partials2 = nullptr;
    int nb2 = 0;
    void *d_desc = nullptr;
    mhd::TileEnt *d_tiles = nullptr;
    mhd::TileEnt *d_tiles_w = nullptr;
    void *h_stage = nullptr;
    size_t h_stage_bytes = 0;
    hipEvent_t stage_evt = nullptr;
    int64_t rcount = 0;      // records written on the device since the last drain
    double clock_hz = 1e8;   // rate of the device wall clock in the records
    std::vector<mhd_diag> host_diag;
    std::vector<double> unit[3];   // cos, sin of 2 pi m / n per axis (forcing phase tables)
    // magnetic spectrum workspace (allocated by the first mhd_spectrum call)
    void *spec_ws = nullptr;
    size_t spec_bytes = 0;
};

namespace mhd {

mhd_status check_params(const mhd_params *p);
mhd_status check_forcing(const mhd_forcing &f);
// filled: other runs of a batch fill the chip, so a grid need not take the tile that
// gives it enough work-groups alone (it takes the z-marching tile where it can)
int default_shape(const mhd_params &p, bool aligned = true, bool filled = false);
bool shape_eligible(const mhd_params &p, int shape, bool aligned);
bool shape_fits(const mhd_params &p, int shape);
int forcing_stride(const mhd_params &p);
int run_ntiles(const mhd_params &p, int shape);
void run_tiles(const mhd_params &p, int shape, int run, std::vector<TileEnt> &out);
// the 64-wide z-marching tiles of substeps 1 and 2 (shapes with `wide`)
void run_tiles_wide(const mhd_params &p, int run, std::vector<TileEnt> &out);
int run_ntiles_wide(const mhd_params &p);
std::vector<TileEnt> xcd_order(const std::vector<TileEnt> &nat);
size_t ctx_footprint(const mhd_params &p);
mhd_status ctx_init(mhd_ctx *c, const mhd_params *p, void *stream, void *const *bufs, int shape);
void ctx_release(mhd_ctx *c);
mhd_status ctx_step(mhd_ctx *c, int64_t n);
mhd_status ctx_drain(mhd_ctx *c);
mhd_status ctx_init_seed(mhd_ctx *c, uint64_t seed, double amp);
mhd_status ctx_forcing_blocks(mhd_ctx *c, int64_t n0, int64_t m, void *dst);
mhd_forcing random_forcing(double kf, double f0, double sigma, uint64_t seed, int64_t n);

template <typename T>
void fill_desc(const mhd_ctx *c, RunDesc<T> &d, int parity0, int64_t step0, const T *forcing, double *records,
               double *partials, int first_tile);
template <typename T>
hipError_t launch_substep(int shape, bool fit, int kind, const RunDesc<T> *runs, const TileEnt *tiles, int ntiles,
                          const TileEnt *wtiles, int nwtiles, int step, hipStream_t st);
template <typename T>
hipError_t launch_finalize(const RunDesc<T> *runs, int nruns, int max_nb2, int step, hipStream_t st);
int run_nb2(const mhd_params &p, int shape);
int x_shift(const mhd_params &p, int shape);
int march_segment(const mhd_params &p, int shape);
int zm_segment(const mhd_params &p);
int shape_fallback(int shape);

}  // namespace mhd
