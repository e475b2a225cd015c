// k_nd_pair.hip -- two colours of the nodal Gauss-Seidel sweep in one pass.
//
// The nodal smoother updates four colours of nodes, by (i mod 2, j mod 2),
// one after another (k_nodal.hip).  The two colours of one row parity share
// their rows, and a node of the second of them depends on nodes of the first
// only in its own row, one node along x and one plane along z (a face of a
// cell spans x and z).  Rows of the other parity are not touched by either
// colour.  So one pass can update both colours of every row of one parity:
// each wavefront owns whole rows (nx = 256, 128, 64 or 32 nodes on 64, 64,
// 32 or 16 lanes, 4 or 2 nodes per lane, x neighbours across the lanes of a
// row by rotation) and marches along z, updating the first colour on plane
// k+1 and then the second on plane k.  No data moves between wavefronts, so
// there is no barrier and no LDS.
//
// A chunk of planes [z0, z1) starts two planes early and ends one late: the
// first colour is recomputed on planes z0-1 and z1 (from old values, as the
// neighbouring chunk computes them) and not stored.  The pass therefore reads
// the iterate it updates from one array and writes another: the first pass of
// a sweep reads rows of both parities from xo and writes its rows to xn; the
// second reads its own rows from xo and the rows just updated from xn, and
// writes its rows to xn, which then holds the whole sweep.  Each node is
// evaluated with the operands and operation order of the one-colour column
// kernel (node_sums order: cells by z, y, x offset; in each cell the three
// face-diagonal corners, then the far corner), so two passes equal four
// colour passes bit for bit.  FP32, periodic x and y.
#include "mp_blk.h"
#include "mp_device.h"
#include "mp_kernels.h"

namespace mp {

bool nd_pair_supported(const NDims& d)
{
    return d.px && d.py && (d.mx == 32 || d.mx == 64 || d.mx == 128 || d.mx == 256) && d.my % 2 == 0 && d.mz >= 2;
}

// Register slots of one wavefront: plane p of the chunk in slot
// (p - z0 + 2) mod NS (node values of rows j-1, j, j+1; sigma of the cell rows
// below and above row j; b of row j).  Compile-time slot names keep values
// in place (see k_fsweep.hip).
template <typename T, int M, int NS>
struct NpCol {
    Strip<T, M> xl[NS], xo[NS], xh[NS], sl[NS], sh[NS], b[NS];
};

// The 2M node values of a row strip with the value just left (q = -1, the
// previous lane's last) and just right (q = 2M, the next lane's first).
template <typename T, int M>
struct Ext {
    T v[2 * M + 2];  // v[q + 1]
};

// Rotations within a row of LPR lanes (a wavefront holds 64 / LPR rows):
// lane l receives lane l - 1 (prev) or l + 1 (next) of its row, wrapping.
// 64: wave rotation (DPP); 16: row rotation (DPP row_ror); 32: ds_bpermute.
template <int LPR>
__device__ __forceinline__ float row_prev(float v)
{
    if constexpr (LPR == 64) {
        return from_prev(v);
    } else if constexpr (LPR == 16) {
        return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x121, 0xf, 0xf, false));
    } else {
        static_assert(LPR == 32, "rows of 16, 32 or 64 lanes");
        const int l = (int)(threadIdx.x & (kWave - 1));
        return __int_as_float(__builtin_amdgcn_ds_bpermute(((l & 32) | ((l + 31) & 31)) << 2, __float_as_int(v)));
    }
}
template <int LPR>
__device__ __forceinline__ float row_next(float v)
{
    if constexpr (LPR == 64) {
        return from_next(v);
    } else if constexpr (LPR == 16) {
        return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x12F, 0xf, 0xf, false));
    } else {
        static_assert(LPR == 32, "rows of 16, 32 or 64 lanes");
        const int l = (int)(threadIdx.x & (kWave - 1));
        return __int_as_float(__builtin_amdgcn_ds_bpermute(((l & 32) | ((l + 1) & 31)) << 2, __float_as_int(v)));
    }
}

template <typename T, int M, int LPR>
__device__ __forceinline__ Ext<T, M> ext(const Strip<T, M>& s)
{
    Ext<T, M> e;
    e.v[0] = row_prev<LPR>(s.v[2 * M - 1]);
#pragma unroll
    for (int q = 0; q < 2 * M; q++) e.v[q + 1] = s.v[q];
    e.v[2 * M + 1] = row_next<LPR>(s.v[0]);
    return e;
}

// One node update at strip position q of row j: rows (r = 0: j-1, 1: j,
// 2: j+1) of the planes below (lo), at (mid) and above (hi) the node, sigma of
// the cells below (cl) and above (ch) in the cell rows below (index 0) and
// above (1) row j.  Node_sums order.
template <typename T, int M>
__device__ __forceinline__ T np_update(int q, const Ext<T, M> (&lo)[3], const Ext<T, M> (&mid)[3],
                                       const Ext<T, M> (&hi)[3], const Ext<T, M> (&cl)[2], const Ext<T, M> (&ch)[2],
                                       T bq, T h12)
{
    T a1 = T(0), a2 = T(0);
#pragma unroll
    for (int oz = 0; oz < 2; oz++)
#pragma unroll
        for (int oy = 0; oy < 2; oy++)
#pragma unroll
            for (int ox = 0; ox < 2; ox++) {
                // cell (i - 1 + ox): strip position q - 1 + ox, i.e. Ext index q + ox
                const T se = oz ? ch[oy].v[q + ox] : cl[oy].v[q + ox];
                const int aa = ox * 2, bb = oy * 2;
                const Ext<T, M>(&vc)[3] = oz ? hi : lo;
                // v[bb][aa]: row bb (0: j-1, 2: j+1), x offset aa - 1
                const T sum = ((mid[bb].v[q + aa] + vc[1].v[q + aa]) + vc[bb].v[q + 1]) + vc[bb].v[q + aa];
                a1 += se;
                a2 = fma(se, sum, a2);
            }
    return (a2 + h12 * bq) / (T(4) * a1);
}

template <typename T, int M, int D, int LPR>
struct NpPass {
    static constexpr int NS = D + 4;
    static_assert(D >= 0 && D <= 3, "the plane loop is unrolled for at most 7 slots");
    using S = Strip<T, M>;
    const NDims& d;
    int z0, z1;
    long long sz, csz;
    long long rl, ro, rh;     // node row offsets of rows j-1, j, j+1 (plus the lane's first node)
    long long cl, ch;         // cell row offsets of the cell rows below and above row j (plus lane)
    const T* __restrict__ xo;   // own rows, before the pass
    const T* __restrict__ xnb;  // rows of the other parity
    T* __restrict__ xn;
    const T* __restrict__ b;
    const T* __restrict__ sg;
    T h12;
    int lead;   // x parity of the first colour
    bool live;  // the lane's row lies inside the grid (else it only loads)

    // node plane P: in range (or wrapped when periodic), else zeros; the load
    // itself is always issued, at a clamped plane
    __device__ __forceinline__ bool node_ok(int P) const { return d.pz || (P >= 0 && P <= d.nz); }
    __device__ __forceinline__ int node_plane(int P) const
    {
        if (d.pz) return P < 0 ? P + d.nz : (P >= d.nz ? P - d.nz : P);
        return P < 0 ? 0 : (P > d.nz ? d.nz : P);
    }
    __device__ __forceinline__ bool cell_ok(int C) const { return d.pz || (C >= 0 && C < d.nz); }
    __device__ __forceinline__ int cell_plane(int C) const
    {
        if (d.pz) return C < 0 ? C + d.nz : (C >= d.nz ? C - d.nz : C);
        return C < 0 ? 0 : (C >= d.nz ? d.nz - 1 : C);
    }
    __device__ __forceinline__ S masked(const S& s, bool ok) const
    {
        S r;
#pragma unroll
        for (int q = 0; q < 2 * M; q++) r.v[q] = ok ? s.v[q] : T(0);
        return r;
    }
    // node plane P into slot Q (rows j-1, j, j+1)
    template <int Q>
    __device__ __forceinline__ void ld_nodes(NpCol<T, M, NS>& s, int P) const
    {
        const long long o = (long long)node_plane(P) * sz;
        const bool ok = node_ok(P);
        s.xl[Q] = masked(ld_strip<T, M>(xnb, o + rl), ok);
        s.xo[Q] = masked(ld_strip<T, M>(xo, o + ro), ok);
        s.xh[Q] = masked(ld_strip<T, M>(xnb, o + rh), ok);
    }
    // cell plane C (sigma) and node plane C (b of row j) into slot Q
    template <int Q>
    __device__ __forceinline__ void ld_cells(NpCol<T, M, NS>& s, int C) const
    {
        const long long o = (long long)cell_plane(C) * csz;
        const bool ok = cell_ok(C);
        s.sl[Q] = masked(ld_strip<T, M>(sg, o + cl), ok);
        s.sh[Q] = masked(ld_strip<T, M>(sg, o + ch), ok);
        s.b[Q] = ld_strip<T, M>(b, (long long)node_plane(C) * sz + ro);
    }

    // Plane step k (slot P0): first colour on node plane k+1, second on k.
    template <int P0>
    __device__ __forceinline__ void step(NpCol<T, M, NS>& s, int k) const
    {
        constexpr int PM = (P0 + NS - 1) % NS, P1 = (P0 + 1) % NS, P2 = (P0 + 2) % NS;
        constexpr int PL = (P0 + 2 + D) % NS, PB = (P0 + 1 + D) % NS;
        ld_nodes<PL>(s, min(k + 2 + D, z1 + 1));
        ld_cells<PB>(s, min(k + 1 + D, z1));
        // first colour on plane k+1: planes k, k+1, k+2; cells k, k+1
        if (node_ok(k + 1)) {
            const Ext<T, M> lo[3] = {ext<T, M, LPR>(s.xl[P0]), ext<T, M, LPR>(s.xo[P0]), ext<T, M, LPR>(s.xh[P0])};
            const Ext<T, M> mid[3] = {ext<T, M, LPR>(s.xl[P1]), ext<T, M, LPR>(s.xo[P1]), ext<T, M, LPR>(s.xh[P1])};
            const Ext<T, M> hi[3] = {ext<T, M, LPR>(s.xl[P2]), ext<T, M, LPR>(s.xo[P2]), ext<T, M, LPR>(s.xh[P2])};
            const Ext<T, M> cb[2] = {ext<T, M, LPR>(s.sl[P0]), ext<T, M, LPR>(s.sh[P0])};
            const Ext<T, M> ca[2] = {ext<T, M, LPR>(s.sl[P1]), ext<T, M, LPR>(s.sh[P1])};
            S out = s.xo[P1];
            if (lead == 0) {
#pragma unroll
                for (int q = 0; q < 2 * M; q += 2) out.v[q] = np_update<T, M>(q, lo, mid, hi, cb, ca, s.b[P1].v[q], h12);
            } else {
#pragma unroll
                for (int q = 1; q < 2 * M; q += 2) out.v[q] = np_update<T, M>(q, lo, mid, hi, cb, ca, s.b[P1].v[q], h12);
            }
            s.xo[P1] = out;
        }
        // second colour on plane k: planes k-1, k, k+1; cells k-1, k
        if (k >= z0 && node_ok(k)) {
            const Ext<T, M> lo[3] = {ext<T, M, LPR>(s.xl[PM]), ext<T, M, LPR>(s.xo[PM]), ext<T, M, LPR>(s.xh[PM])};
            const Ext<T, M> mid[3] = {ext<T, M, LPR>(s.xl[P0]), ext<T, M, LPR>(s.xo[P0]), ext<T, M, LPR>(s.xh[P0])};
            const Ext<T, M> hi[3] = {ext<T, M, LPR>(s.xl[P1]), ext<T, M, LPR>(s.xo[P1]), ext<T, M, LPR>(s.xh[P1])};
            const Ext<T, M> cb[2] = {ext<T, M, LPR>(s.sl[PM]), ext<T, M, LPR>(s.sh[PM])};
            const Ext<T, M> ca[2] = {ext<T, M, LPR>(s.sl[P0]), ext<T, M, LPR>(s.sh[P0])};
            S out = s.xo[P0];
            if (lead == 0) {
#pragma unroll
                for (int q = 1; q < 2 * M; q += 2) out.v[q] = np_update<T, M>(q, lo, mid, hi, cb, ca, s.b[P0].v[q], h12);
            } else {
#pragma unroll
                for (int q = 0; q < 2 * M; q += 2) out.v[q] = np_update<T, M>(q, lo, mid, hi, cb, ca, s.b[P0].v[q], h12);
            }
            s.xo[P0] = out;
            if (live) st_strip<T, M>(xn, (long long)k * sz + ro, out);
        }
    }
};

// Row r = 2 (w * 64 / LPR + lane / LPR) + rowpar for wavefront w (LPR lanes
// per row, nx = 2 M LPR nodes); blocks of four wavefronts; blockIdx.y is the
// plane chunk.
template <typename T, int M, int D, int LPR>
__global__ __launch_bounds__(256) void k_nd_pair(NDims d, int lz, const T* __restrict__ xo,
                                                 const T* __restrict__ xnb, T* __restrict__ xn,
                                                 const T* __restrict__ b, const T* __restrict__ sg, T h12, int rowpar,
                                                 int lead)
{
    using F = NpPass<T, M, D, LPR>;
    constexpr int NS = F::NS;
    constexpr int RPW = kWave / LPR;
    const int lane = threadIdx.x & (kWave - 1);
    const int w = (int)blockIdx.x * (blockDim.x / kWave) + (int)threadIdx.x / kWave;
    if (2 * w * RPW + rowpar >= d.my) return;  // the wavefront's first row is beyond the grid
    int j = 2 * (w * RPW + lane / LPR) + rowpar;
    const bool live = j < d.my;
    if (!live) j = rowpar;  // rows beyond the grid load a row inside it and store nothing
    const int xi = 2 * M * (lane % LPR);
    const int jl = j > 0 ? j - 1 : d.my - 1, jh = j + 1 < d.my ? j + 1 : 0;  // periodic y
    F f{d};
    f.z0 = (int)blockIdx.y * lz;
    f.z1 = min(f.z0 + lz, d.mz);
    f.sz = (long long)d.mx * d.my;
    f.csz = (long long)d.nx * d.ny;
    f.rl = (long long)jl * d.mx + xi;
    f.ro = (long long)j * d.mx + xi;
    f.rh = (long long)jh * d.mx + xi;
    f.cl = (long long)jl * d.nx + xi;  // cell row j-1: between node rows j-1 and j
    f.ch = (long long)j * d.nx + xi;   // cell row j: between node rows j and j+1
    f.xo = xo;
    f.xnb = xnb;
    f.xn = xn;
    f.b = b;
    f.sg = sg;
    f.h12 = h12;
    f.lead = lead;
    f.live = live;

    const int zs = f.z0 - 2;
    NpCol<T, M, NS> s;
#pragma unroll
    for (int q = 0; q < NS; q++) s.xl[q] = s.xo[q] = s.xh[q] = s.sl[q] = s.sh[q] = s.b[q] = zero_strip<T, M>();
    // node planes zs .. zs+D+1, cell planes (and b) zs .. zs+D
    f.template ld_nodes<0>(s, zs);
    f.template ld_nodes<1 % NS>(s, zs + 1);
    if constexpr (D >= 1) f.template ld_nodes<2 % NS>(s, zs + 2);
    if constexpr (D >= 2) f.template ld_nodes<3 % NS>(s, zs + 3);
    if constexpr (D >= 3) f.template ld_nodes<4 % NS>(s, zs + 4);
    f.template ld_cells<0>(s, zs);
    if constexpr (D >= 1) f.template ld_cells<1 % NS>(s, zs + 1);
    if constexpr (D >= 2) f.template ld_cells<2 % NS>(s, zs + 2);
    if constexpr (D >= 3) f.template ld_cells<3 % NS>(s, zs + 3);
    int k = zs;
    for (; k + NS <= f.z1; k += NS) {
        f.template step<0>(s, k);
        f.template step<1>(s, k + 1);
        f.template step<2>(s, k + 2);
        f.template step<3>(s, k + 3);
        if constexpr (NS > 4) f.template step<4 % NS>(s, k + 4);
        if constexpr (NS > 5) f.template step<5 % NS>(s, k + 5);
        if constexpr (NS > 6) f.template step<6 % NS>(s, k + 6);
    }
    if (k < f.z1) f.template step<0>(s, k);
    if (k + 1 < f.z1) f.template step<1>(s, k + 1);
    if (k + 2 < f.z1) f.template step<2>(s, k + 2);
    if constexpr (NS > 4)
        if (k + 3 < f.z1) f.template step<3 % NS>(s, k + 3);
    if constexpr (NS > 5)
        if (k + 4 < f.z1) f.template step<4 % NS>(s, k + 4);
    if constexpr (NS > 6)
        if (k + 5 < f.z1) f.template step<5 % NS>(s, k + 5);
}

namespace {

constexpr int kNpAhead = 1;
constexpr int kNpMinPlanes = 3;

// Planes per chunk: the shortest (at least kNpMinPlanes) for which the grid
// is resident at once, lengthened until its plane steps are whole groups of
// the unrolled loop.  Short chunks read four extra planes each, but from L2:
// at 256 x 256 nodes the resident grid wins over longer chunks.
template <typename T, int M, int LPR>
int np_chunk(const NDims& d, long long gx)
{
    constexpr int NS = kNpAhead + 4;
    static int resident = 0;
    if (resident == 0) {
        int dev = 0, ncu = 0, per_cu = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu,
                                                         reinterpret_cast<const void*>(k_nd_pair<T, M, kNpAhead, LPR>),
                                                         256, 0) != hipSuccess)
            return 13;
        resident = max(1, ncu * max(per_cu, 1));
    }
    const long long chunks = max(1LL, resident / gx);
    int lz = max((int)((d.mz + chunks - 1) / chunks), kNpMinPlanes);
    lz += (NS - (lz + 2) % NS) % NS;
    return lz;
}

template <typename T, int M, int LPR>
void np_launch(const NDims& d, const T* xo, const T* xnb, T* xn, const T* b, const T* sg, T h12, int rowpar,
               int lead, hipStream_t s)
{
    const int rows = (d.my - rowpar + 1) / 2;
    const int per_block = 4 * (kWave / LPR);
    const long long gx = (rows + per_block - 1) / per_block;
    const int lz = np_chunk<T, M, LPR>(d, gx);
    const dim3 grid((unsigned)gx, (unsigned)((d.mz + lz - 1) / lz));
    hipLaunchKernelGGL((k_nd_pair<T, M, kNpAhead, LPR>), grid, dim3(256), 0, s, d, lz, xo, xnb, xn, b, sg, h12,
                       rowpar, lead);
}

}  // namespace

template <typename T>
void launch_nd_pair(const NDims& d, const T* xo, const T* xnb, T* xn, const T* b, const T* sg, T h12, int rowpar,
                    int lead, hipStream_t s)
{
    switch (d.mx) {
    case 256: np_launch<T, 2, 64>(d, xo, xnb, xn, b, sg, h12, rowpar, lead, s); break;
    case 128: np_launch<T, 1, 64>(d, xo, xnb, xn, b, sg, h12, rowpar, lead, s); break;
    case 64: np_launch<T, 1, 32>(d, xo, xnb, xn, b, sg, h12, rowpar, lead, s); break;
    default: np_launch<T, 1, 16>(d, xo, xnb, xn, b, sg, h12, rowpar, lead, s); break;
    }
}

template void launch_nd_pair<float>(const NDims&, const float*, const float*, float*, const float*, const float*,
                                    float, int, int, hipStream_t);

}  // namespace mp
