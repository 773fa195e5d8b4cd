// fdlb_internal.h -- types shared by the HIP kernels and the host runtime of libfdlb.
//
// Layout in HBM (per instance, per buffer slot h = 0, 1 -- the ping-pong halves -- and, for
// contexts that take two steps per pass, h = 2, the intermediate step's buffer):
//   f[h]  : 33 planes of ny rows x fpitch elements (float64 or float32), structure of
//           arrays, x fastest; plane q = 0 is the rest particle, q = 1 + 8(k-1) + (i-1) the
//           velocity of speed k and direction i pi/4 (Eq. dvm_eq_1).  In the deviation
//           layout (PREC_DEV) the planes hold g_q = f_q - f^eq_q(M) in float32.
//   P[h]  : pressure n T of every cell, ny rows x ppitch float64.
//   M[h]  : moments (n, ux, uy, T) of every cell, 4 planes of ny rows x ppitch float64,
//           written by the step that produced the distributions and read by the next
//           (ppitch == fpitch, so one element offset addresses a cell in both).
//   PW[h] : 4 rows of wlen float64, the pressure of the mirror image of the cells next to
//           each reflecting side (x-, x+, y-, y+), read by the switching function.
// A single step reads slot h and writes slot 1 - h; a two-step pass reads h, keeps the
// intermediate step of its tiles in LDS (and in slot 2 where single-step tiles need it) and
// writes 1 - h.  Kernels take the slots packed as io = in | out << 4.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fdlb {

constexpr int NQ = 33;
constexpr int BC_PERIODIC = 0, BC_OUTFLOW = 1, BC_DIRICHLET = 2, BC_WALL = 3;
constexpr int PREC_F64 = 0, PREC_F32 = 1, PREC_DEV = 2;

// Per-instance constants and buffer pointers.  Lives in device memory and is read with
// uniform (scalar) loads.  All constants are float64, computed on the host in a fixed
// order (see fdlb_api.cpp).
struct Inst {
    int32_t nx, ny, fpitch, ppitch;
    int64_t fplane;          // elements per f plane (ny * fpitch)
    int32_t bc[4];           // x-, x+, y-, y+
    int32_t wlen, prec;
    void *f[3];
    double *P[3];
    double *M[3];
    double *PW[3];
    int64_t mplane;          // elements per moment plane (ny * ppitch)
    int32_t *flag;           // sticky non-physical flag (shared by a batch)
    double th0;              // theta of line IV = lam |dP / sum P| + th0: 0 with Eq. (add4);
                             // the frozen value (lam = 0) when theta is frozen (Sec. 4)
    double v[4], vs[4];      // speeds and speed * sqrt(2)/2 (diagonal components)
    double eax[4], edg[4];   // |v|^2 / 2 for axis and diagonal velocities
    double FA[4], FB[4], FC[4], Fden[4]; // weight polynomial constants, Eq. (fk_eq1)
    double k1[2][2][4], k2[2][2][4], k3[2][2][4]; // [alpha][axis=0, diag=1][speed], c >= 0
    double kk[2][2][4];                           // k1 + 2 k3 (the deviation update's weight)
    double dt, dx, dy, dtau, lam;
    double Fdinv[4];         // 1 / Fden (deviation path, which needs no fixed order)
    double cdx, cdy;         // dt / dx, dt / dy
    float kf[3][2][2][4];    // float copies of k1, k2, k3 (float32 path)
    float kkf[2][2][4];      // k1 + 2 k3, float32 path
    float vf[4], vsf[4];     // float copies of v and vs
    // Dirichlet data per slot: slots 0..3 the sides, 4..7 their lower segments
    double bcstate[8][4];    // (rho, ux, uy, T)
    double bcf[8][NQ];       // ghost vectors (values representable in storage)
    double bcP[8];           // their pressures
    // lower segments: ghost cells at centre coordinate (i + 1/2) d < split0 + split1 * t
    // along side s take condition bclo[s] (BC_PERIODIC: no lower segment)
    int32_t bclo[4];
    double split0[4], split1[4];
    const int64_t *clock;    // steps since the state was set (time of the moving segments)
};

struct Tile {
    int32_t inst, x0, y0, flags;  // flags: kTileRing for two-step tiles beside single-step ones
};
// A two-step tile whose x or y neighbour takes single steps: it also stores its intermediate
// step (values and moments) in slot 2, where that neighbour's second step reads it.
constexpr int32_t kTileRing = 1;

// Packed input / output buffer slots of a step launch.
__host__ __device__ constexpr int io_pack(int in, int out) { return in | (out << 4); }
__host__ __device__ constexpr int io_in(int io) { return io & 15; }
__host__ __device__ constexpr int io_out(int io) { return io >> 4; }

struct TileShape {
    int tx, ty;
};

// Tile shapes the step kernel is instantiated for (index = shape id - 1).
constexpr TileShape kTileShapes[] = {{32, 8}, {64, 4}, {16, 16}, {64, 8}, {16, 4}, {128, 4}, {32, 4}, {16, 8}};
constexpr int kNumTileShapes = sizeof(kTileShapes) / sizeof(kTileShapes[0]);

// Host-side launchers (fdlb_kernels.hip).  `insts` / `tiles` are device pointers.
// kind: 0 interior tiles, 1 tube tiles (periodic height == tile height), 2 edge tiles, all
// one step per launch; 3 two-step tiles (float64, shape kTwoStepShape, their tile and four
// cells around it inside the grid), two steps per launch
constexpr int kNumTileKinds = 4;
constexpr int kKindTwoStep = 3;
#ifndef FDLB_TWO_STEP_SHAPE
#define FDLB_TWO_STEP_SHAPE 7
#endif
constexpr int kTwoStepShape = FDLB_TWO_STEP_SHAPE;  // 16 x 8: two blocks per CU
hipError_t launch_step(int prec, int shape, int kind, const Inst *insts, const Tile *tiles, int ntiles, int io,
                       hipStream_t s);
// Two steps of the float64 two-step tiles: reads slot io_in, writes slot io_out (and slot 2
// for ring tiles).
hipError_t launch_step2(const Inst *insts, const Tile *tiles, int ntiles, int io, hipStream_t s);
int tile_kind(int x0, int y0, int tx, int ty, int nx, int ny, int bc_y);
// Plain copy of the stored planes of `tiles` (interior tiles) from half `half` to the other.
hipError_t launch_plane_copy(int prec, int shape, const Inst *insts, const Tile *tiles, int ntiles, int half,
                             hipStream_t s);
hipError_t launch_bc_setup(int prec, Inst *insts, int inst, hipStream_t s);
hipError_t launch_fill(int prec, const Inst *insts, int inst, int nx, int ny, const double *fields, int half,
                       hipStream_t s);
hipError_t launch_derive(int prec, const Inst *insts, int inst, int nx, int ny, int half, hipStream_t s);
hipError_t launch_moments(int prec, const Inst *insts, int inst, int nx, int ny, int half, double *out,
                          hipStream_t s);
hipError_t launch_diag(int prec, const Inst *insts, int inst, int nx, int ny, int half, double *partials,
                       int npart_offset, hipStream_t s);
hipError_t launch_diag_final(const double *partials, int nparts, double *sums, hipStream_t s);
// Partial blocks (of 256 cells) the fixed scratch of the allocation-free diagnostics holds:
// 2^16 blocks, 2^24 cells over all instances of a context (2 MiB of float64 partials).
constexpr int kDiagScratchParts = 1 << 16;
// Device address of that scratch on the current device (hipGetSymbolAddress).
hipError_t diag_scratch_address(double **ptr);
hipError_t launch_tick(int64_t *clock, hipStream_t s);
// Float64 edge tiles run the streaming body (FDLB_STREAM_EDGE=0: the register-resident
// body, which writes the wall-image pressures itself).
#ifndef FDLB_STREAM_EDGE
#define FDLB_STREAM_EDGE 1
#endif
// Pressures of the mirror images beside reflecting sides from the distributions of half
// `half`, for the k instances (maxlen: the longest side); after each float64 step when
// FDLB_STREAM_EDGE is on.
hipError_t launch_wall_pressure(const Inst *insts, int k, int maxlen, int half, hipStream_t s);
int diag_blocks(int nx, int ny);

}  // namespace fdlb
