// mp_launch.h -- launch-shape helpers shared by the kernel files.
#pragma once
#include <hip/hip_runtime.h>

namespace mp {

inline int pow2_at_least(int n, int cap)
{
    int p = 1;
    while (p < n && p < cap) p <<= 1;
    return p;
}

// Block and grid covering an nx x ny x nz box with up to 256 threads per
// block, x fastest (64 lanes along x when nx allows), no index division.
struct Shape3 {
    dim3 grid, block;
};

inline Shape3 cells3(int nx, int ny, int nz)
{
    const int bx = pow2_at_least(nx, 64);
    const int by = pow2_at_least(ny, 256 / bx);
    const int bz = pow2_at_least(nz, 256 / (bx * by));
    Shape3 s;
    s.block = dim3(bx, by, bz);
    s.grid = dim3((nx + bx - 1) / bx, (ny + by - 1) / by, (nz + bz - 1) / bz);
    return s;
}

// z-marching launch: blocks of bx x by columns, each column walks lz planes.
struct ShapeZ {
    dim3 grid, block;
    int lz;
    long long blocks() const { return (long long)grid.x * grid.y * grid.z; }
};

// Always 256 threads per block (full wavefronts, which the block reductions
// need); columns outside the grid are masked by the kernels.
inline ShapeZ zmarch(int nx, int ny, int nz, long long max_blocks)
{
    const int bx = pow2_at_least(nx, 64);
    const int by = 256 / bx;
    ShapeZ s;
    s.block = dim3(bx, by, 1);
    const long long cols = (long long)((nx + bx - 1) / bx) * ((ny + by - 1) / by);
    int lz = 4;
    while (lz < nz && cols * ((nz + lz - 1) / lz) > max_blocks) lz <<= 1;
    if (lz > nz) lz = nz;
    s.lz = lz;
    s.grid = dim3((nx + bx - 1) / bx, (ny + by - 1) / by, (nz + lz - 1) / lz);
    return s;
}

}  // namespace mp
