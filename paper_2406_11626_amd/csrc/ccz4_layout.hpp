// Layout constants and small helpers shared by the host planner and the device kernels.
#pragma once
#include <cstdint>

namespace ccz4 {

constexpr int NV = 59;          // 58 first-order variables + K_0
constexpr int NEVOL = 58;       // evolved slots
constexpr int PN = 9;           // interior cells per axis
constexpr int HL = 3;           // halo layers per face
constexpr int NBX = 15;         // box cells per axis
constexpr int XS = 16;          // padded row length (doubles)
constexpr int YS = XS;          // y stride
constexpr int ZS = NBX * XS;    // z stride (240)
constexpr int CS = NBX * ZS;    // slot stride (3600)
constexpr int64_t PS = (int64_t)NV * CS; // patch stride (212400 doubles)
constexpr int NCELL = PN * PN * PN;      // 729 interior cells
constexpr int NFACE = 3 * PN * PN;       // 243 cells per face slab

// slot map of the first-order variables
__host__ __device__ constexpr int sym(int i, int j)
{
    return i <= j ? (i == 0 ? j : (i == 1 ? 2 + j : 5)) : (j == 0 ? i : (j == 1 ? 2 + i : 5));
}
constexpr int SG = 0, SALPHA = 6, SBETA = 7, SPHI = 10, SAT = 11, SK = 17, STHETA = 18,
              SGHAT = 19, SBB = 22, SA = 25, SB = 28, SD = 37, SP = 55, SK0 = 58;
// the auxiliaries A, B, D, P (slots 25..57): evolved in the first-order formulation,
// reconstructed from the primaries in the second-order one
__host__ __device__ constexpr bool aux_slot(int v) { return v >= SA && v < SK0; }

// box offset of cell (x, y, z) inside one slot of a patch
__host__ __device__ constexpr int boff(int x, int y, int z) { return z * ZS + y * YS + x; }

// Accumulator of the fused RK4 stage: state-sized, but private to that stage and laid out for
// whole-line access.  Within one slot of a patch, interior cell i (0..242) of z-slab sl (cell
// (x, y, z) with i = ((z - 3 - 3 sl) * 9 + y - 3) * 9 + x - 3) sits at 256 sl + i, so the lanes of
// a wave cover consecutive 128-byte lines; ghost cell idx of the Sommerfeld face (axis, side)
// sits at 768 + (2 axis + (side > 0)) * 243 + idx.
constexpr int ACC_SLAB = 256;
constexpr int ACC_GHOST = 3 * ACC_SLAB;
static_assert(ACC_SLAB >= NFACE && ACC_GHOST + 6 * NFACE <= CS, "accumulator layout must fit a slot");
__host__ __device__ constexpr int acc_cell(int sl, int i) { return ACC_SLAB * sl + i; }
__host__ __device__ constexpr int acc_ghost(int axis, int side, int idx)
{
    return ACC_GHOST + (2 * axis + (side > 0 ? 1 : 0)) * NFACE + idx;
}

// face-task kinds of the halo fill
enum FaceKind : int32_t { FK_COPY = 0, FK_NEUMANN = 1, FK_RESTRICT = 2, FK_PROLONG = 3 };

struct FaceTask {
    int32_t kind;
    int32_t patch;     // destination leaf
    int32_t axis;      // 0, 1, 2
    int32_t side;      // -1 or +1
    int32_t src[9];    // COPY: src[0]; RESTRICT: 9 fine leaves [u2*3+u1]; PROLONG: src[0] coarse leaf
    int32_t o1, o2;    // PROLONG: position of the fine patch inside the coarse face
};

enum RegridKind : int32_t { RG_COPY = 0, RG_PROLONG = 1, RG_RESTRICT = 2 };

struct RegridTask {  // how one leaf of a new mesh takes its data from the old mesh
    int32_t kind;
    int32_t src;       // COPY: old leaf; PROLONG: old parent leaf
    int32_t o[3];      // PROLONG: position of the new leaf inside the parent (0..2 per axis)
    int32_t kid[27];   // RESTRICT: the 27 old leaves, index (z/3)*9 + (y/3)*3 + x/3
};

struct BoundaryFace {  // a Sommerfeld face of a leaf and its background slab
    int32_t patch, axis, side, bg;
};

struct PatchGeom {
    double org[3];     // lower corner of the interior
    double dx[3];
    int32_t level, pad;
};

// A leaf's cube and its parent's cube (lower corner and edge lengths, the parent's only for
// level >= 1), for refinement tags by coordinates
struct TrackBox {
    double lo[3], L[3], plo[3], pL[3];
    int32_t level, pad;
};

// Slots sampled by tracers (passed by value)
struct TracerSlots {
    int32_t n;
    int32_t v[NV];
};

// Leaf lookup of points: the domain's lower corner, the cube edge of the finest level present and
// that level.  A point's cube index at the finest level, floor((x - org) / fine), decides the leaf
// of every level (passed by value).
struct LeafLookup {
    double org[3];
    double fine[3];
    int32_t top, pad;
};

// Per-level radii of tracker-based refinement (passed by value)
constexpr int MAX_TRACK_LEVELS = 16;
struct TrackRadii {
    int32_t n;
    double r[MAX_TRACK_LEVELS];
};

}  // namespace ccz4
