// gfx950 kernels of the IB-LB wetting solver.
//
// Every kernel works on a batch of independent droplets described by a
// device table of DropDev records; a single droplet is a batch of one.
//
//   k_lb              fused pull-stream + BGK collide + Guo source for every
//                     fluid cell (eq. LBE, equilibrium, S_i, moments of eqs.
//                     hydro_var1/hydro_var2); HBM bound, one cell per lane
//   k_force_spread    nodal surface-tension + wetting forces, spread to the
//                     lattice with the Peskin 4-point kernel (eq. force_spread)
//   k_interp_advect   lattice velocity interpolated at the nodes (eq.
//                     vel_interpolation) and forward-Euler advection
//   k_ib_fused2       2D: interpolation and advection of one step fused with
//                     the forces and spreading of the next
//   k_force3,
//   k_spread3         3D: forces one lane per vertex (surface tension, an
//                     elastic interface's shear part, wetting), then
//                     spreading summed per chunk of nearby vertices in LDS
//   k_cross2,
//   k_cross3          crossings of the interface with the lattice rows, for
//                     the inside/outside classification of two viscosities
//   k_inside_mask     that classification as a per-cell mask
//   k_tri_ref         reference triangles of an elastic interface
//   k_cell_sums,
//   k_diag, k_contact FP64 reductions for the diagnostics and the contact
//                     radius
//
// Populations are stored as deviations f_i - w_i (see lattice.hpp), in two
// ping-pong buffers laid out [i][z][y][x] per droplet, x fastest.
//
// The force density F and the velocity U are dense per-cell arrays, but the
// lattice kernel touches them only inside the interface band: the spreading
// kernel raises a one-byte flag for every x strip (8 or 16 cells, see
// Strip) that receives a tap, and only the cells of flagged strips read F, write U for the
// interpolation and clear F (where it is not zero already).  The spread F is accumulated in fixed point (64-bit integers of
// 2^-40 force units, see fq_of), so its value does not depend on the order
// in which the nodes' contributions arrive; a prescribed force field is kept
// in fp32 in an array of its own.  The flags come in two sets, one per step parity: a lattice
// update reads its own parity's set and clears the other one for the
// spreading of the next step.
#pragma once

#include <hip/hip_runtime.h>
#include <limits.h>
#include <stdint.h>

#include <type_traits>

#include "lattice.hpp"

namespace iblb {

constexpr int kBlock = 256;   // threads per block of every kernel
// Cells per band flag: 8 (an eighth of a wavefront) for 2D lattices in
// 16-bit storage, 16 (a quarter) otherwise.  With 8-cell strips the fp16
// 256-droplet 2D batch's lattice kernel took 121.8 against 128.2 us per
// launch, while the fp32 1024x512 D2Q9 step took 13.68 against 13.48 us and
// the 3D benchmark step 255.9 against 255.0 us.  A row's flags are padded to
// a multiple of the strips of 64 cells, so that a tiled wavefront (64 cells
// of one row, starting at a multiple of 64) finds its strips' flags in one
// aligned word (64 bits for 8-cell strips, 32 for 16-cell ones).  The node
// kernels take the width from the droplet record (DropDev::sshift).
template <int DIM, int S>
struct Strip {
    static constexpr int shift = (DIM == 2 && S != ST_F32) ? 3 : 4;
    static constexpr int n = 1 << shift;
    static constexpr int per64 = 64 >> shift;  // strips of 64 cells (bytes of a word)
    using Word = typename std::conditional<per64 == 8, uint64_t, uint32_t>::type;
};

struct DropDev {
    int nx, ny, nz, nstrip;
    int sshift;           // log2 of the cells per band flag (see Strip)
    int bcx, bcy, bcz, ncell;
    long long f_off;      // element offset of the populations (Q arrays, fst apart)
    long long c_off;      // cell offset; vector arrays start at dim * c_off
    long long flag_off;   // byte offset of the band flags
    float omega, guo;     // 1/tau and 1 - 1/(2 tau)
    int force_mode;       // 0: immersed boundary, 1: prescribed field
    int active;
    int node_off, n_nodes;
    int tri_off, n_tris;
    int tile_off, n_tiles;  // this droplet's run in the list of all tiles
    int wetting, n_exp, m_exp;
    int fst;              // element stride between population arrays (>= ppl nz)
    int ppl;              // elements per z-plane of a population array (>= nx ny):
                          // cell (x, y, z) sits at z ppl + y nx + x
    double sigma, A, xi, zcut;
    // two viscosities (viscosity ratio != 1): cells enclosed by the
    // interface relax with omega_in / guo_in
    int visc;
    int row_off;          // first lattice row (z * ny + y) of this droplet in the crossing tables
    float omega_in, guo_in;
    double win[3];        // classification window [win, win + n) of each axis
    double img_base, img_r;  // x image of cell centre c: c + img_base (+ nx if c < img_r)
    double shear;         // surface shear modulus of an elastic interface (0: liquid)
    double respace;       // rate beta of the tangential re-spacing of a 2D outline (0: off)
};

struct DiagDev {
    double mass_dev;            // sum over cells of rho - 1
    double mom[3];
    double sum_F[3];
    double sum_phi[3];
    double dropped[3];
    double volume, area;
    double min_h, max_h;
    double max_un, max_u;
    double edge_min, edge_max;
    double cross_lo, cross_hi;  // 2D: outermost crossings of y = zcut
    double cross_r;             // 3D: mean distance of crossings to their centre
    double cross_n;
};

// Fixed-point accumulation of the spread force density (eq. force_spread):
// every contribution phi_j Delta is rounded to an integer number of 2^-40
// force units and added with a 64-bit integer atomic.  Integer addition is
// associative, so the sum, and the fp32 value the lattice kernel forms from
// it (one rounding of the exact sum), are the same whatever order the
// contributions arrive in.  A contribution must stay below 2^10 in
// magnitude (then up to 2^12 of them cannot overflow a cell); a larger or
// non-finite one means the run has blown up: it is dropped and the
// droplet flagged unstable (status bit 2).
constexpr double kFqScale = 1099511627776.0;  // 2^40
constexpr float kFqMax = 1024.f;
__device__ __forceinline__ bool fq_ok(float v) { return fabsf(v) < kFqMax; }  // NaN: false
__device__ __forceinline__ unsigned long long fq_of(float v) {
    return (unsigned long long)(long long)rint((double)v * kFqScale);
}
__device__ __forceinline__ float fq_value(unsigned long long v) {
    return (float)((double)(long long)v * (1.0 / kFqScale));
}

// One cell's collision in deviation form (eqs. LBE, f^eq, S_i,
// hydro_var1/2), in two parts so that callers can store each population as
// soon as it is relaxed: Moments takes the streamed deviations f_i - w_i and
// the force (half-force velocity); relax() gives post-collision population
// i: BGK towards the second-order equilibrium plus the Guo source.
template <int DIM>
struct Moments {
    float drho, rho, ux, uy, uz, usq, uF, Fx, Fy, Fz;
    __device__ __forceinline__ Moments(const float* f, float fx, float fy, float fz) : Fx(fx), Fy(fy), Fz(fz) {
        using L = Lattice<DIM>;
        float jx = 0.f, jy = 0.f, jz = 0.f;
        drho = 0.f;
#pragma unroll
        for (int i = 0; i < L::Q; ++i) {
            drho += f[i];
            if (L::c[i][0] > 0) jx += f[i]; else if (L::c[i][0] < 0) jx -= f[i];
            if (L::c[i][1] > 0) jy += f[i]; else if (L::c[i][1] < 0) jy -= f[i];
            if (DIM == 3) { if (L::c[i][2] > 0) jz += f[i]; else if (L::c[i][2] < 0) jz -= f[i]; }
        }
        rho = 1.f + drho;
        const float inv = 1.f / rho;
        ux = (jx + 0.5f * Fx) * inv;
        uy = (jy + 0.5f * Fy) * inv;
        uz = DIM == 3 ? (jz + 0.5f * Fz) * inv : 0.f;
        usq = ux * ux + uy * uy + uz * uz;
        uF = ux * Fx + uy * Fy + uz * Fz;
    }
    __device__ __forceinline__ float relax(int i, float fi, float om, float g, bool forced) const {
        using L = Lattice<DIM>;
        const int cx = L::c[i][0], cy = L::c[i][1], cz = L::c[i][2];
        const float cu = cx * ux + cy * uy + (DIM == 3 ? cz * uz : 0.f);
        // f_eq - w = w (rho - 1) + w rho (3 cu + 4.5 cu^2 - 1.5 u^2)
        const float feq = L::w[i] * (drho + rho * (3.f * cu + 4.5f * cu * cu - 1.5f * usq));
        float v = fi - om * (fi - feq);
        if (forced) {
            const float cF = cx * Fx + cy * Fy + (DIM == 3 ? cz * Fz : 0.f);
            // S_i = (1 - 1/2tau) w_i [3 (c - U).F + 9 (c.U)(c.F)]
            v += g * L::w[i] * (3.f * (cF - uF) + 9.f * cu * cF);
        }
        return v;
    }
};

// ---------------------------------------------------------------------------
// Cells enclosed by the interface (viscosity ratio != 1)
// ---------------------------------------------------------------------------
// The cells inside the closed interface relax with their own tau (Sec.
// IB-LB, last paragraph).  They are found by casting a ray along +x through
// every lattice row (the cell centres of one y, z): the node kernels record,
// per row, the x at which the interface crosses the row's line, and a cell
// is inside when an odd number of crossings lies beyond its centre.  The
// interface is not wrapped across periodic boundaries: rows and cell
// centres are taken at their periodic image inside the droplet's window
// [win, win + n) of each axis, centred on the mean of the node positions.
// Crossing tables: a count per row and kCrossCap x values per row, one pair
// of tables per step parity.
constexpr int kCrossCap = 16;

__device__ __forceinline__ bool cell_inside(const DropDev& D, const int* __restrict__ cnt,
                                            const double* __restrict__ xs, int x, int row) {
    const long long r = (long long)D.row_off + row;
    int n = cnt[r];
    n = n < kCrossCap ? n : kCrossCap;
    const double c = (double)x + 0.5;
    const double xi = c + D.img_base + (c < D.img_r ? (double)D.nx : 0.0);
    bool in = false;
    for (int k = 0; k < n; ++k) in ^= xs[r * kCrossCap + k] > xi;
    return in;
}

// ---------------------------------------------------------------------------
// Lattice kernel
// ---------------------------------------------------------------------------
// NT = 1 writes the new populations with non-temporal stores (fp32 ones
// with sc1 as well, see nt_store_policy): they are not read again before
// the next launch, so they need not displace cached lines.
// NTL = 1 reads the populations with non-temporal loads: each is read once
// per launch (neighbouring wavefronts share only the edges of the lines
// that x-streamed populations straddle).
// VIS = 1 (instantiated only while some droplet of the handle has two
// viscosities) takes each cell's relaxation time from the classification.
// BX = 0 is the flat form: a block takes 256 consecutive cells of the
// droplet in storage order, whatever nx is, so rows that are not a multiple
// of 64 cells long leave no lanes idle (a wavefront may then span two rows,
// and the band flag and the row of the classification are read per lane).
// ONE = 1 (a handle holding a single droplet) reads that droplet's
// parameters without waiting for the block's tile entry, so the two loads
// that open every wavefront are in flight together.
template <int DIM, int S, int BX, int NT, int NTL, int VIS, int ONE>
__global__ __launch_bounds__(kBlock) void k_lb(const DropDev* __restrict__ drops,
                                               const int4* __restrict__ tiles,
                                               const typename Codec<S>::T* __restrict__ fsrc_all,
                                               typename Codec<S>::T* __restrict__ fdst_all,
                                               const float* __restrict__ F_all,
                                               unsigned long long* __restrict__ Fq_all,
                                               float* __restrict__ U_all,
                                               float* __restrict__ rho_all,
                                               float* __restrict__ Fout_all,
                                               const uint8_t* __restrict__ flags_all,
                                               uint8_t* __restrict__ flags_clr, int full,
                                               const int* __restrict__ xcnt,
                                               const double* __restrict__ xpos,
                                               int* __restrict__ xclr) {
    using L = Lattice<DIM>;
    using C = Codec<S>;
    constexpr int Q = L::Q;
    constexpr bool FLAT = BX == 0;
    constexpr int BY = FLAT ? 1 : kBlock / (FLAT ? 1 : BX);
    const int4 tile = tiles[blockIdx.x];  // the host lays the list out in block order
    const DropDev& D = drops[ONE ? 0 : tile.x];
    const int nx = D.nx, ny = D.ny, nz = D.nz;
    int x, y, z;
    if constexpr (FLAT) {
        const int c = tile.y * kBlock + (int)threadIdx.x;
        if (c >= D.ncell) return;
        const int r = c / nx;
        x = c - r * nx;
        z = r / ny;
        y = r - z * ny;
    } else {
        x = tile.y * BX + (int)(threadIdx.x % (FLAT ? 1 : BX));
        y = tile.z * BY + (int)(threadIdx.x / (FLAT ? 1 : BX));
        z = tile.w;
        if (x >= nx || y >= ny) return;
    }
    const int ncell = D.ncell, fst = D.fst, ppl = D.ppl;
    const int cell = (z * ny + y) * nx + x;  // field arrays
    const int pc = z * ppl + y * nx + x;      // population arrays
    const typename C::T* __restrict__ fsrc = fsrc_all + D.f_off;
    typename C::T* __restrict__ fdst = fdst_all + D.f_off;

    // source coordinates for c = +1 (xm) and c = -1 (xp); -1 marks a wall
    int xm = x - 1, xp = x + 1, ym = y - 1, yp = y + 1, zm = z - 1, zp = z + 1;
    if (xm < 0) xm = D.bcx ? -1 : nx - 1;
    if (xp >= nx) xp = D.bcx ? -1 : 0;
    if (ym < 0) ym = D.bcy ? -1 : ny - 1;
    if (yp >= ny) yp = D.bcy ? -1 : 0;
    if (DIM == 3) {
        if (zm < 0) zm = D.bcz ? -1 : nz - 1;
        if (zp >= nz) zp = D.bcz ? -1 : 0;
    }

    // the band flag of this cell's strip is requested before the
    // populations: loads return in order, so waiting for the flag then does
    // not wait for the populations, and a band wavefront's F loads overlap
    // them instead of following them
    // A tiled wavefront reads its strips' flags as one aligned word.
    using SW = typename Strip<DIM, S>::Word;
    constexpr int SPW = Strip<DIM, S>::per64;
    const long long fi = D.flag_off + (long long)(z * ny + y) * D.nstrip + (x >> Strip<DIM, S>::shift);
    int flag;
    if constexpr (FLAT) {
        flag = D.force_mode == 1 ? 1 : (int)flags_all[fi];
    } else {
        const SW w = D.force_mode == 1 ? ~SW(0) : *reinterpret_cast<const SW*>(flags_all + (fi & ~(long long)(SPW - 1)));
        flag = (int)((w >> (8 * (int)(fi & (SPW - 1)))) & 0xffu);
    }
    // Populations move through buffer instructions (32-bit lane offsets,
    // base in scalar registers): one descriptor per opposite pair (i,
    // opp(i)), based at the lower index, so that a lane offset never
    // exceeds 2 fst elements and a bounce-back read of opp(i) stays inside
    // the same descriptor.  Q fst < 2^31 elements keeps every offset and
    // size below 2^31 bytes.
    constexpr int SB = storage_bytes<S>();
    float f[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const int cx = L::c[i][0], cy = L::c[i][1], cz = L::c[i][2];
        const int sx = cx > 0 ? xm : (cx < 0 ? xp : x);
        const int sy = cy > 0 ? ym : (cy < 0 ? yp : y);
        const int sz = DIM == 3 ? (cz > 0 ? zm : (cz < 0 ? zp : z)) : 0;
        // a source beyond a wall means the population was reflected there:
        // take the opposite population of this cell (half-way bounce-back)
        const bool wall = (sx | sy | sz) < 0;
        const int lo = i == 0 ? 0 : ((i & 1) ? i : i - 1);
        const auto rs = buffer_of(fsrc + (long long)lo * fst, (i == 0 ? 1 : 2) * fst * SB);
        const int rel = wall ? (opp(i) - lo) * fst + pc : (i - lo) * fst + sz * ppl + sy * nx + sx;
        f[i] = C::template load_buf<NTL ? kBufNT : 0>(rs, (unsigned)rel * SB);
    }

    const float* __restrict__ F = F_all + (long long)DIM * D.c_off;
    unsigned long long* __restrict__ Fq = Fq_all + (long long)DIM * D.c_off;
    float* __restrict__ U = U_all + (long long)DIM * D.c_off;
    // band: this lane's strip is flagged (band); a wavefront holding any
    // band lane adds the Guo source on every lane (exactly zero where F is)
    bool band, forced;
    float Fx = 0.f, Fy = 0.f, Fz = 0.f;
    unsigned long long q0 = 0, q1 = 0, q2 = 0;
    if (D.force_mode == 1) {
        band = forced = true;
    } else {
        // band flags of this step (set by the spreading); those of the
        // other parity, read by the step before, are cleared for the
        // spreading of the next step by the first lane of each strip
        band = flag != 0;
        forced = __builtin_amdgcn_ballot_w64(band) != 0;
        if constexpr (FLAT) {
            if (flags_clr && (x & (Strip<DIM, S>::n - 1)) == 0) flags_clr[fi] = 0;
        } else {
            if (flags_clr && (x & 63) == 0) *reinterpret_cast<SW*>(flags_clr + fi) = SW(0);
        }
    }
    if (band) {
        if (D.force_mode == 1) {
            Fx = F[cell];
            Fy = F[ncell + cell];
            if (DIM == 3) Fz = F[2 * ncell + cell];
        } else {
            q0 = Fq[cell];
            q1 = Fq[ncell + cell];
            if (DIM == 3) q2 = Fq[2 * ncell + cell];
            Fx = fq_value(q0);
            Fy = fq_value(q1);
            Fz = fq_value(q2);
        }
    }
    const Moments<DIM> M(f, Fx, Fy, Fz);
    const float rho = M.rho, ux = M.ux, uy = M.uy, uz = M.uz;
    float om = D.omega, g = D.guo;
    if (VIS && D.visc) {
        // every lane of a wavefront lies in the same row when BX >= 64
        const int row = FLAT ? z * ny + y : __builtin_amdgcn_readfirstlane(z * ny + y);
        if (cell_inside(D, xcnt, xpos, x, row)) {
            om = D.omega_in;
            g = D.guo_in;
        }
        // the other parity's table was read by the previous step: clear it
        // for the crossings of the next step
        if (x == 0 && xclr) xclr[D.row_off + row] = 0;
    }
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const float fn = M.relax(i, f[i], om, g, forced);
        const int lo = i == 0 ? 0 : ((i & 1) ? i : i - 1);
        const auto rd = buffer_of(fdst + (long long)lo * fst, (i == 0 ? 1 : 2) * fst * SB);
        C::template store_buf<NT ? nt_store_policy<S>() : 0>(rd, (unsigned)((i - lo) * fst + pc) * SB, fn);
    }

    if (band && D.force_mode == 0) {
        // interface band: keep U for the interpolation, hand back a clean F
        U[cell] = ux;
        U[ncell + cell] = uy;
        if (DIM == 3) U[2 * ncell + cell] = uz;
        if (q0) Fq[cell] = 0;
        if (q1) Fq[ncell + cell] = 0;
        if (DIM == 3 && q2) Fq[2 * ncell + cell] = 0;
    }
    if (full) {
        float* __restrict__ Fo = Fout_all + (long long)DIM * D.c_off;
        rho_all[D.c_off + cell] = rho;
        U[cell] = ux;
        U[ncell + cell] = uy;
        Fo[cell] = Fx;
        Fo[ncell + cell] = Fy;
        if (DIM == 3) {
            U[2 * ncell + cell] = uz;
            Fo[2 * ncell + cell] = Fz;
        }
    }
}

// Nodes whose coordinates are not finite or lie absurdly far from any box
// (|q| > 2^24) are never turned into tap indices: converting such a value to
// int is undefined and could yield an index far outside the lattice.  The
// kernels skip the node and flag its droplet unstable instead.
constexpr double kFarCoord = 16777216.0;
__device__ __forceinline__ bool coord_ok(double v) { return fabs(v) <= kFarCoord; }  // NaN: false

// Cell index of tap base + k along an axis of n cells: wrapped on a periodic
// axis, -1 beyond a wall.  base comes from a coordinate that passed coord_ok,
// so base + k cannot overflow.
__device__ __forceinline__ int tap_index(int base, int k, int n, int wall) {
    int i = base + k;
    if (i >= 0 && i < n) return i;
    if (wall) return -1;
    i %= n;
    return i < 0 ? i + n : i;
}

struct NodeArrays {
    const double* pos;   // [3][stride]
    double* pos_w;       // positions of the next step, written by the advection
    float* phi;          // [3][stride]
    float* qdot;         // [3][stride]
    float* dropped;      // [3][stride]
    const int* node_drop;
    const int* tri;      // [3][tstride] global node ids
    const int* inc;      // incidence entries (triangle << 2 | slot)
    const int* inc_beg;
    const int* inc_end;
    const int* perm;     // node ids in spatial (Morton) order, per droplet
    const double* tref;  // [5][tstride] reference triangles of elastic interfaces
    int stride, tstride, ntot;
};

__device__ __forceinline__ double ipow(double s, int n) {
    double p = 1.0;
    for (int k = 0; k < n; ++k) p *= s;
    return p;
}

// Pi(h) of eq. (disjoin-p)
__device__ __forceinline__ double wetting_pi(const DropDev& D, double h) {
    const double s = D.xi / h;
    return D.A * (ipow(s, D.n_exp) - ipow(s, D.m_exp));
}

// Geometry of a node of a 2D closed CCW polygon from its own position q
// and those of its ring neighbours qm (previous) and qp (next):
// surface-tension force sigma (t_j - t_{j-1}), node normal (mean of the
// adjacent outward edge normals), node length chi = l_{j-1} + l_j.
__device__ __forceinline__ void geom_2d(double sigma, const double qm[2], const double q[2],
                                        const double qp[2], double fs[2], double n[2],
                                        double& chi) {
    const double ex = qp[0] - q[0], ey = qp[1] - q[1];
    const double fx = q[0] - qm[0], fy = q[1] - qm[1];
    const double le = sqrt(ex * ex + ey * ey);
    const double lf = sqrt(fx * fx + fy * fy);
    fs[0] = sigma * (ex / le - fx / lf);
    fs[1] = sigma * (ey / le - fy / lf);
    double nx = ey / le + fy / lf, ny = -ex / le - fx / lf;
    const double nn = sqrt(nx * nx + ny * ny);
    n[0] = nx / nn;
    n[1] = ny / nn;
    chi = le + lf;
}

__device__ __forceinline__ void ring_2d(const DropDev& D, int j, int& jm, int& jp) {
    const int N = D.n_nodes, loc = j - D.node_off;
    jm = D.node_off + (loc == 0 ? N - 1 : loc - 1);
    jp = D.node_off + (loc == N - 1 ? 0 : loc + 1);
}

// Tangential re-spacing of a 2D outline, an addition to the method for long
// runs (a line tension has no tangential stiffness, so nodes carried by the
// fluid drift along the outline and open gaps): node m with ring neighbours
// a and b moves by beta/2 (|q_b - q_m| - |q_m - q_a|) along the unit chord
// q_b - q_a, computed from the positions before the advection and added to
// the advected position.  Uniform spacing is left alone.
__device__ __forceinline__ void respace_move(double beta, const double qa[3], const double qm[3],
                                             const double qb[3], double dq[2]) {
    const double lm = sqrt((qm[0] - qa[0]) * (qm[0] - qa[0]) + (qm[1] - qa[1]) * (qm[1] - qa[1]));
    const double lp = sqrt((qb[0] - qm[0]) * (qb[0] - qm[0]) + (qb[1] - qm[1]) * (qb[1] - qm[1]));
    const double cx = qb[0] - qa[0], cy = qb[1] - qa[1];
    const double c = sqrt(cx * cx + cy * cy);
    const double sc = c > 0.0 ? 0.5 * beta * (lp - lm) / c : 0.0;
    dq[0] = sc * cx;
    dq[1] = sc * cy;
}

__device__ __forceinline__ void node_geom_2d(const DropDev& D, const NodeArrays& A, int j,
                                             double q[2], double fs[2], double n[2],
                                             double& chi) {
    int jm, jp;
    ring_2d(D, j, jm, jp);
    const int st = A.stride;
    const double qm[2] = {A.pos[jm], A.pos[st + jm]}, qp[2] = {A.pos[jp], A.pos[st + jp]};
    q[0] = A.pos[j];
    q[1] = A.pos[st + j];
    geom_2d(D.sigma, qm, q, qp, fs, n, chi);
}

// Elastic interface: the shear part w_s = mu_s (b + 1 - e^a) of the strain
// energy, with the invariants a = (1/2) log det G, b = (1/2) tr G - 1 of
// eq. strain_inv (G = F^T F shares the nonzero eigenvalues of D D^T).  The
// in-plane deformation gradient of triangle t is F = [e1 e2] Ei, Ei the
// inverse of its reference edges in a frame of the reference plane (stored
// with the reference area A0 by k_tri_ref).  With d(a)/dF = F G^-1 and
// d(b)/dF = F the energy gradient is dW/dF = A0 mu_s (F - e^a F G^-1);
// dW/dF Ei^T holds dW/dq1 and dW/dq2 in its columns and
// dW/dq0 = -(dW/dq1 + dW/dq2).  Adds -dW/dq of the triangle's slot s to fs.
__device__ __forceinline__ void shear_force(double mu, const NodeArrays& A, int t, int s,
                                            const double e1[3], const double e2[3], double fs[3]) {
    const int ts = A.tstride;
    const double Ei[2][2] = {{A.tref[t], A.tref[ts + t]}, {A.tref[2 * ts + t], A.tref[3 * ts + t]}};
    const double A0 = A.tref[4 * ts + t];
    double F[3][2];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        F[k][0] = e1[k] * Ei[0][0] + e2[k] * Ei[1][0];
        F[k][1] = e1[k] * Ei[0][1] + e2[k] * Ei[1][1];
    }
    const double g00 = F[0][0] * F[0][0] + F[1][0] * F[1][0] + F[2][0] * F[2][0];
    const double g01 = F[0][0] * F[0][1] + F[1][0] * F[1][1] + F[2][0] * F[2][1];
    const double g11 = F[0][1] * F[0][1] + F[1][1] * F[1][1] + F[2][1] * F[2][1];
    const double det = g00 * g11 - g01 * g01;
    const double ea = sqrt(det);
    const double i00 = g11 / det, i01 = -g01 / det, i11 = g00 / det;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const double d0 = A0 * mu * (F[k][0] - ea * (F[k][0] * i00 + F[k][1] * i01));
        const double d1 = A0 * mu * (F[k][1] - ea * (F[k][0] * i01 + F[k][1] * i11));
        const double g1 = d0 * Ei[0][0] + d1 * Ei[0][1];
        const double g2 = d0 * Ei[1][0] + d1 * Ei[1][1];
        fs[k] += s == 0 ? g1 + g2 : (s == 1 ? -g1 : -g2);
    }
}

// Contribution of triangle t (vertices P, node j in slot s) to node j: the
// surface-tension force -sigma/2 n_t x (q_c - q_b) (the gradient of sigma
// times the triangle's area), its unit normal and its area; plus the shear
// part of an elastic interface.
__device__ __forceinline__ void tri_contrib(const DropDev& D, const NodeArrays& A, int t, int s,
                                            const double P[3][3], double fs[3], double ns[3],
                                            double& chi) {
    const double e1[3] = {P[1][0] - P[0][0], P[1][1] - P[0][1], P[1][2] - P[0][2]};
    const double e2[3] = {P[2][0] - P[0][0], P[2][1] - P[0][1], P[2][2] - P[0][2]};
    double nt[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2],
                    e1[0] * e2[1] - e1[1] * e2[0]};
    const double len = sqrt(nt[0] * nt[0] + nt[1] * nt[1] + nt[2] * nt[2]);
    nt[0] /= len;
    nt[1] /= len;
    nt[2] /= len;
    const int sb = s == 2 ? 0 : s + 1, sc = s == 0 ? 2 : s - 1;
    const double d[3] = {P[sc][0] - P[sb][0], P[sc][1] - P[sb][1], P[sc][2] - P[sb][2]};
    fs[0] -= 0.5 * D.sigma * (nt[1] * d[2] - nt[2] * d[1]);
    fs[1] -= 0.5 * D.sigma * (nt[2] * d[0] - nt[0] * d[2]);
    fs[2] -= 0.5 * D.sigma * (nt[0] * d[1] - nt[1] * d[0]);
    ns[0] += nt[0];
    ns[1] += nt[1];
    ns[2] += nt[2];
    chi += 0.5 * len;
    if (D.shear != 0.0) shear_force(D.shear, A, t, s, e1, e2, fs);
}

// Incident triangles of a vertex fetched in one batch (icosphere and cap
// meshes have 5-6 per vertex; a vertex with more takes the plain loop).
constexpr int kIncBatch = 8;

// Geometry of vertex j of a closed 3D triangle mesh (CCW seen from
// outside): surface-tension force -sigma d(area)/dq_j summed over the
// incident triangles, vertex normal (mean of the incident unit normals),
// chi = sum of the incident areas.
__device__ __forceinline__ void node_geom_3d(const DropDev& D, const NodeArrays& A, int j,
                                             double q[3], double fs[3], double n[3],
                                             double& chi) {
    const int st = A.stride, ts = A.tstride;
    q[0] = A.pos[j];
    q[1] = A.pos[st + j];
    q[2] = A.pos[2 * st + j];
    fs[0] = fs[1] = fs[2] = 0.0;
    double ns[3] = {0.0, 0.0, 0.0};
    chi = 0.0;
    const int beg = A.inc_beg[j], end = A.inc_end[j];
    if (end > beg && end - beg <= kIncBatch) {
        // the usual vertex (at most kIncBatch triangles): the incidence
        // entries, then the triangles' vertex ids, then the positions of the
        // two other vertices of each are each fetched in one batch, three
        // round trips in all instead of three per triangle; out-of-range
        // slots repeat the last entry and are not summed
        const int cnt = end - beg;
        int e[kIncBatch];
#pragma unroll
        for (int i = 0; i < kIncBatch; ++i) e[i] = A.inc[beg + (i < cnt ? i : cnt - 1)];
        int vb[kIncBatch], vc[kIncBatch];
#pragma unroll
        for (int i = 0; i < kIncBatch; ++i) {
            const int t = e[i] >> 2, s = e[i] & 3;
            const int sb = s == 2 ? 0 : s + 1, sc = s == 0 ? 2 : s - 1;
            vb[i] = A.tri[sb * ts + t];
            vc[i] = A.tri[sc * ts + t];
        }
        double Pb[kIncBatch][3], Pc[kIncBatch][3];
#pragma unroll
        for (int i = 0; i < kIncBatch; ++i)
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                Pb[i][a] = A.pos[a * st + vb[i]];
                Pc[i][a] = A.pos[a * st + vc[i]];
            }
#pragma unroll
        for (int i = 0; i < kIncBatch; ++i) {
            if (i >= cnt) break;
            const int t = e[i] >> 2, s = e[i] & 3;
            const int sb = s == 2 ? 0 : s + 1;
            // vertex slot s of triangle t is node j itself
            double P[3][3];
#pragma unroll
            for (int m = 0; m < 3; ++m)
#pragma unroll
                for (int a = 0; a < 3; ++a) P[m][a] = m == s ? q[a] : (m == sb ? Pb[i][a] : Pc[i][a]);
            tri_contrib(D, A, t, s, P, fs, ns, chi);
        }
        const double nn = sqrt(ns[0] * ns[0] + ns[1] * ns[1] + ns[2] * ns[2]);
        n[0] = ns[0] / nn;
        n[1] = ns[1] / nn;
        n[2] = ns[2] / nn;
        return;
    }
    for (int k = beg; k < end; ++k) {
        const int e = A.inc[k];
        const int t = e >> 2, s = e & 3;
        const int v0 = A.tri[t], v1 = A.tri[ts + t], v2 = A.tri[2 * ts + t];
        double P[3][3];
        const int vv[3] = {v0, v1, v2};
#pragma unroll
        for (int m = 0; m < 3; ++m) {
            P[m][0] = A.pos[vv[m]];
            P[m][1] = A.pos[st + vv[m]];
            P[m][2] = A.pos[2 * st + vv[m]];
        }
        tri_contrib(D, A, t, s, P, fs, ns, chi);
    }
    const double nn = sqrt(ns[0] * ns[0] + ns[1] * ns[1] + ns[2] * ns[2]);
    n[0] = ns[0] / nn;
    n[1] = ns[1] / nn;
    n[2] = ns[2] / nn;
}

// ---------------------------------------------------------------------------
// Node kernels: one lane per (node, tap)
// ---------------------------------------------------------------------------
// A node owns a group of TAPS consecutive lanes (16 in 2D: 4 nodes per
// wavefront; 64 in 3D: one wavefront per node).  Every lane of the group
// evaluates the node's geometry (same instructions, broadcast loads), then
// handles one tap of the delta kernel; sums over the taps are shuffles
// inside the group.  This turns a serial chain of 16 or 64 scattered
// memory operations per thread into one per lane.
// Droplet of node j.  ONE: the handle holds a single droplet, so the index
// is a compile-time 0 and its record is read through the scalar cache
// instead of per lane after a lookup.
template <bool ONE>
__device__ __forceinline__ int node_droplet(const NodeArrays& A, int j) {
    return ONE ? 0 : A.node_drop[j];
}

// Workgroup size of the node kernels that give each node a group of tap
// lanes (the groups never straddle a wavefront).  One wavefront per
// workgroup spreads the few thousand lanes of a droplet's nodes over four
// times as many compute units as 256-lane workgroups; measured 1.4% faster
// per coupled 1024x512 step, the same in 3D.
#ifndef IBLB_NODE_BLOCK
#define IBLB_NODE_BLOCK 64
#endif
constexpr int kNodeBlock = IBLB_NODE_BLOCK;


template <int DIM>
struct Taps {
    static constexpr int n = DIM == 2 ? 16 : 64;
};

// Lanes per node of the interpolation kernel: one per tap in 2D; in 3D two
// taps per lane, so the 64 taps of a vertex take half a wavefront and a
// batch of vertices half as many wavefronts.
template <int DIM>
struct InterpLanes {
    static constexpr int n = DIM == 3 ? Taps<3>::n / 2 : Taps<2>::n;
};

// ---------------------------------------------------------------------------
// Peskin 4-point kernel
// ---------------------------------------------------------------------------
// For a node at coordinate q the four taps are the cells base..base+3 with
// base = floor(q - 1/2) - 1, at distances 1 + r, r, 1 - r, 2 - r from the
// node (r = q - 1/2 - floor(q - 1/2) in [0, 1)).  With s = sqrt(1 + 4r - 4r^2)
// both branches of Psi reduce to
//   Psi(1+r) = (3 - 2r - s)/8, Psi(r) = (3 - 2r + s)/8,
//   Psi(1-r) = (1 + 2r + s)/8, Psi(2-r) = (1 + 2r - s)/8,
// so one square root serves all four taps.
//
// peskin_tap: weight of tap k (0..3) of a node at coordinate q, and the
// index of tap 0.
__device__ __forceinline__ float peskin_tap(double q, int k, int& base) {
    const double u = q - 0.5;
    const double fl = floor(u);
    const float r = (float)(u - fl);
    base = (int)fl - 1;
    const float s = sqrtf(1.f + 4.f * r * (1.f - r));
    const float a = k < 2 ? 3.f - 2.f * r : 1.f + 2.f * r;
    return (a + ((k == 1 || k == 2) ? s : -s)) * 0.125f;
}

template <int G>
__device__ __forceinline__ float group_sum(float v) {
#pragma unroll
    for (int o = G / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Lattice cell of this lane's tap, or -1 when it falls beyond a wall; also
// the tap's row (z * ny + y) and x for the band flag.
template <int DIM>
__device__ __forceinline__ int lane_tap(const DropDev& D, const double q[3], int k, float& w,
                                        int& row, int& ix) {
    int bx, by, bz = 0;
    w = peskin_tap(q[0], k & 3, bx) * peskin_tap(q[1], (k >> 2) & 3, by);
    if (DIM == 3) w *= peskin_tap(q[2], k >> 4, bz);
    ix = tap_index(bx, k & 3, D.nx, D.bcx);
    const int iy = tap_index(by, (k >> 2) & 3, D.ny, D.bcy);
    const int iz = DIM == 3 ? tap_index(bz, k >> 4, D.nz, D.bcz) : 0;
    if ((ix | iy | iz) < 0) return -1;
    row = iz * D.ny + iy;
    return row * D.nx + ix;
}

// This lane's tap of the spreading of nodal force ph at q (eq.
// force_spread); with want_dropped the group's wall losses are summed and
// stored by lane 0.
template <int DIM>
__device__ __forceinline__ void spread_lane(const DropDev& D, const NodeArrays& A, int j, int k,
                                            const double q[3], const float ph[3],
                                            unsigned long long* __restrict__ Fq_all,
                                            uint8_t* __restrict__ flags_all, int want_dropped,
                                            int* __restrict__ status_d) {
    constexpr int T = Taps<DIM>::n;
    float w;
    int row, ix;
    const int cell = lane_tap<DIM>(D, q, k, w, row, ix);
    float lost[3] = {0.f, 0.f, 0.f};
    if (cell < 0) {
#pragma unroll
        for (int a = 0; a < DIM; ++a) lost[a] = ph[a] * w;
    } else {
        unsigned long long* __restrict__ Fq = Fq_all + (long long)DIM * D.c_off;
        bool fine = true;
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            const float v = ph[a] * w;
            if (fq_ok(v))
                atomicAdd(Fq + a * D.ncell + cell, fq_of(v));
            else
                fine = false;
        }
        if (!fine) atomicOr(status_d, 2);
        flags_all[D.flag_off + row * D.nstrip + (ix >> D.sshift)] = 1;
    }
    if (want_dropped) {
#pragma unroll
        for (int a = 0; a < DIM; ++a) lost[a] = group_sum<T>(lost[a]);
        if (k == 0)
#pragma unroll
            for (int a = 0; a < DIM; ++a) A.dropped[a * A.stride + j] = lost[a];
    }
}

// ---------------------------------------------------------------------------
// Nodal forces + spreading (eq. force_spread)
// ---------------------------------------------------------------------------
template <int DIM, bool ONE>
__global__ __launch_bounds__(kNodeBlock) void k_force_spread(const DropDev* __restrict__ drops,
                                                         NodeArrays A,
                                                         unsigned long long* __restrict__ Fq_all,
                                                         uint8_t* __restrict__ flags_all,
                                                         int* __restrict__ status,
                                                         int want_dropped) {
    constexpr int T = Taps<DIM>::n;
    const int gid = blockIdx.x * kNodeBlock + threadIdx.x;
    const int j = gid / T, k = gid % T;
    if (j >= A.ntot) return;
    const int d = node_droplet<ONE>(A, j);
    const DropDev& D = drops[d];
    if (!D.active || D.force_mode != 0) return;
    double q[3] = {0, 0, 0}, fs[3] = {0, 0, 0}, n[3] = {0, 0, 0}, chi;
    double share;
    if (DIM == 2) {
        node_geom_2d(D, A, j, q, fs, n, chi);
        share = 0.5 * chi;
    } else {
        node_geom_3d(D, A, j, q, fs, n, chi);
        share = chi / 3.0;
    }
    if (D.wetting) {
        const double P = wetting_pi(D, q[DIM - 1]);
#pragma unroll
        for (int a = 0; a < DIM; ++a) fs[a] -= share * P * n[a];
    }
    float ph[3] = {0.f, 0.f, 0.f};
#pragma unroll
    for (int a = 0; a < DIM; ++a) ph[a] = (float)fs[a];
    if (k == 0)
#pragma unroll
        for (int a = 0; a < DIM; ++a) A.phi[a * A.stride + j] = ph[a];
    bool ok = true;
#pragma unroll
    for (int a = 0; a < DIM; ++a) ok &= coord_ok(q[a]);
    if (!ok) {  // the whole group leaves together
        if (k == 0) atomicOr(status + d, 4);
        return;
    }
    spread_lane<DIM>(D, A, j, k, q, ph, Fq_all, flags_all, want_dropped, status + d);
}

// Nodes that do not move this step (droplet inactive, prescribed force
// field, or non-finite input) still carry their positions into the buffer
// of the next step.
template <int DIM>
__device__ __forceinline__ void hold_position(const NodeArrays& A, int j, int k) {
    if (k < DIM) A.pos_w[k * A.stride + j] = A.pos[k * A.stride + j];
}

// ---------------------------------------------------------------------------
// Crossings of the interface with the lattice rows (see cell_inside)
// ---------------------------------------------------------------------------
// Record a crossing of droplet row r (z * ny + y) at x.  More than
// kCrossCap crossings on one row set status bit 8.
__device__ __forceinline__ void add_crossing(const DropDev& D, int* __restrict__ cnt,
                                             double* __restrict__ xs, int r, double x,
                                             int* __restrict__ status, int d) {
    const long long rr = (long long)D.row_off + r;
    const int slot = atomicAdd(cnt + rr, 1);
    if (slot < kCrossCap)
        xs[rr * kCrossCap + slot] = x;
    else
        atomicOr(status + d, 8);
}

// Whether a node lies inside the droplet's classification window along its
// periodic axes (along a wall axis the box itself bounds it).  A node
// outside would make the rows' crossings miss or double the interface: the
// crossing kernels then set status bit 16.
template <int DIM>
__device__ __forceinline__ bool in_window(const DropDev& D, const double* q) {
    bool ok = true;
    if (!D.bcx) ok = ok && q[0] >= D.win[0] && q[0] < D.win[0] + D.nx;
    if (!D.bcy) ok = ok && q[1] >= D.win[1] && q[1] < D.win[1] + D.ny;
    if (DIM == 3 && !D.bcz) ok = ok && q[2] >= D.win[2] && q[2] < D.win[2] + D.nz;
    return ok;
}

// Row index of the image j of a row coordinate along an axis of n rows.
__device__ __forceinline__ int wrap_row(int j, int n) {
    j %= n;
    return j < 0 ? j + n : j;
}

// Edge a -> b of a 2D polygon: crossings with the row lines y = j + 1/2
// inside the window, each edge taken half-open in y so that a line through
// a vertex is crossed once by the two edges that share it.  Coordinates
// have passed coord_ok.
__device__ __forceinline__ void cross_edge_2d(const DropDev& D, int* __restrict__ cnt,
                                              double* __restrict__ xs, const double a[2],
                                              const double b[2], int* __restrict__ status, int d) {
    if (!in_window<2>(D, a)) atomicOr(status + d, 16);  // node a of this edge
    const double wlo = D.win[1], whi = D.win[1] + D.ny;
    const double lo = fmax(fmin(a[1], b[1]), wlo), hi = fmin(fmax(a[1], b[1]), whi);
    if (!(lo <= hi)) return;
    const int j0 = (int)ceil(lo - 0.5), j1 = (int)floor(hi - 0.5);
    for (int j = j0; j <= j1; ++j) {
        const double Y = j + 0.5;
        if ((a[1] <= Y) == (b[1] <= Y) || Y < wlo || Y >= whi) continue;
        const double x = a[0] + (Y - a[1]) * (b[0] - a[0]) / (b[1] - a[1]);
        add_crossing(D, cnt, xs, wrap_row(j, D.ny), x, status, d);
    }
}

// Side of the point (y, z) relative to the directed edge P -> Q of a
// triangle projected onto the y-z plane: the sign of the orientation,
// computed from the edge's endpoints in the order of their node ids so that
// the two triangles sharing an edge evaluate the same number; a zero is
// resolved as for the point moved by (eps, eps^2).  val receives the
// orientation itself (for barycentric weights).
__device__ __forceinline__ int edge_side(const double P[3], int ip, const double Q[3], int iq,
                                         double y, double z, double& val) {
    const bool flip = ip > iq;
    const double* A = flip ? Q : P;
    const double* B = flip ? P : Q;
    const double dy = B[1] - A[1], dz = B[2] - A[2];
    const double o = dy * (z - A[2]) - dz * (y - A[1]);
    int sg = o > 0.0 ? 1 : (o < 0.0 ? -1 : 0);
    if (sg == 0) sg = dz != 0.0 ? (dz > 0.0 ? -1 : 1) : (dy > 0.0 ? 1 : (dy < 0.0 ? -1 : 0));
    val = flip ? -o : o;
    return flip ? -sg : sg;
}

// Triangle (node ids i[3], positions P[3][3]): crossings with the row lines
// (y, z) = (j + 1/2, k + 1/2) inside the window whose projection the
// triangle covers; x by barycentric interpolation.
__device__ __forceinline__ void cross_tri_3d(const DropDev& D, int* __restrict__ cnt,
                                             double* __restrict__ xs, const double P[3][3],
                                             const int id[3], int* __restrict__ status, int d) {
    if (!(in_window<3>(D, P[0]) && in_window<3>(D, P[1]) && in_window<3>(D, P[2])))
        atomicOr(status + d, 16);
    const double ylo = D.win[1], yhi = D.win[1] + D.ny, zlo = D.win[2], zhi = D.win[2] + D.nz;
    const double y0 = fmax(fmin(fmin(P[0][1], P[1][1]), P[2][1]), ylo);
    const double y1 = fmin(fmax(fmax(P[0][1], P[1][1]), P[2][1]), yhi);
    const double z0 = fmax(fmin(fmin(P[0][2], P[1][2]), P[2][2]), zlo);
    const double z1 = fmin(fmax(fmax(P[0][2], P[1][2]), P[2][2]), zhi);
    if (!(y0 <= y1 && z0 <= z1)) return;
    const int j0 = (int)ceil(y0 - 0.5), j1 = (int)floor(y1 - 0.5);
    const int k0 = (int)ceil(z0 - 0.5), k1 = (int)floor(z1 - 0.5);
    for (int k = k0; k <= k1; ++k) {
        const double Z = k + 0.5;
        if (Z < zlo || Z >= zhi) continue;
        for (int j = j0; j <= j1; ++j) {
            const double Y = j + 0.5;
            if (Y < ylo || Y >= yhi) continue;
            double e0, e1, e2;
            const int s0 = edge_side(P[1], id[1], P[2], id[2], Y, Z, e0);
            const int s1 = edge_side(P[2], id[2], P[0], id[0], Y, Z, e1);
            const int s2 = edge_side(P[0], id[0], P[1], id[1], Y, Z, e2);
            if (s0 == 0 || s0 != s1 || s1 != s2) continue;
            const double x = (e0 * P[0][0] + e1 * P[1][0] + e2 * P[2][0]) / (e0 + e1 + e2);
            add_crossing(D, cnt, xs, wrap_row(k, D.nz) * D.ny + wrap_row(j, D.ny), x, status, d);
        }
    }
}

// Crossings of the interfaces at the positions A.pos: of the active
// droplets with two viscosities, or of every droplet with an interface when
// all != 0.  2D: one lane per polygon edge (node j to its ring successor).
template <bool ONE>
__global__ __launch_bounds__(kBlock) void k_cross2(const DropDev* __restrict__ drops, NodeArrays A,
                                                   int* __restrict__ cnt, double* __restrict__ xs,
                                                   int* __restrict__ status, int all) {
    const int j = blockIdx.x * kBlock + threadIdx.x;
    if (j >= A.ntot) return;
    const int d = node_droplet<ONE>(A, j);
    const DropDev& D = drops[d];
    if (D.force_mode != 0 || !(all || (D.active && D.visc))) return;
    int jm, jp;
    ring_2d(D, j, jm, jp);
    const int st = A.stride;
    const double a[2] = {A.pos[j], A.pos[st + j]}, b[2] = {A.pos[jp], A.pos[st + jp]};
    if (!(coord_ok(a[0]) && coord_ok(a[1]) && coord_ok(b[0]) && coord_ok(b[1]))) {
        atomicOr(status + d, 4);
        return;
    }
    cross_edge_2d(D, cnt, xs, a, b, status, d);
}

// 3D: one lane per triangle.
template <bool ONE>
__global__ __launch_bounds__(kBlock) void k_cross3(const DropDev* __restrict__ drops, NodeArrays A,
                                                   int ttot, int* __restrict__ cnt,
                                                   double* __restrict__ xs, int* __restrict__ status,
                                                   int all) {
    const int t = blockIdx.x * kBlock + threadIdx.x;
    if (t >= ttot) return;
    const int ts = A.tstride, st = A.stride;
    const int id[3] = {A.tri[t], A.tri[ts + t], A.tri[2 * ts + t]};
    const int d = node_droplet<ONE>(A, id[0]);
    const DropDev& D = drops[d];
    if (D.force_mode != 0 || !(all || (D.active && D.visc))) return;
    double P[3][3];
    bool ok = true;
#pragma unroll
    for (int m = 0; m < 3; ++m)
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            P[m][a] = A.pos[a * st + id[m]];
            ok = ok && coord_ok(P[m][a]);
        }
    if (!ok) {
        atomicOr(status + d, 4);
        return;
    }
    cross_tri_3d(D, cnt, xs, P, id, status, d);
}

// Stress-free reference of droplet d's triangles for the elastic interface
// (see shear_force), from the positions A.pos, one lane per triangle:
// frame t1 along the first edge, t2 in the triangle's plane; the inverse of
// the reference edge matrix and the reference area.
__global__ __launch_bounds__(kBlock) void k_tri_ref(const DropDev* __restrict__ drops, int d, NodeArrays A,
                                                    double* __restrict__ tref) {
    const DropDev& D = drops[d];
    const int l = blockIdx.x * kBlock + threadIdx.x;
    if (l >= D.n_tris) return;
    const int t = D.tri_off + l, ts = A.tstride, st = A.stride;
    const int v[3] = {A.tri[t], A.tri[ts + t], A.tri[2 * ts + t]};
    double r1[3], r2[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        r1[k] = A.pos[k * st + v[1]] - A.pos[k * st + v[0]];
        r2[k] = A.pos[k * st + v[2]] - A.pos[k * st + v[0]];
    }
    const double l1 = sqrt(r1[0] * r1[0] + r1[1] * r1[1] + r1[2] * r1[2]);
    const double t1[3] = {r1[0] / l1, r1[1] / l1, r1[2] / l1};
    const double n[3] = {r1[1] * r2[2] - r1[2] * r2[1], r1[2] * r2[0] - r1[0] * r2[2],
                         r1[0] * r2[1] - r1[1] * r2[0]};
    double t2[3] = {n[1] * t1[2] - n[2] * t1[1], n[2] * t1[0] - n[0] * t1[2], n[0] * t1[1] - n[1] * t1[0]};
    const double l2 = sqrt(t2[0] * t2[0] + t2[1] * t2[1] + t2[2] * t2[2]);
    t2[0] /= l2;
    t2[1] /= l2;
    t2[2] /= l2;
    const double a = r1[0] * t1[0] + r1[1] * t1[1] + r1[2] * t1[2];
    const double b = r2[0] * t1[0] + r2[1] * t1[1] + r2[2] * t1[2];
    const double c = r1[0] * t2[0] + r1[1] * t2[1] + r1[2] * t2[2];
    const double e = r2[0] * t2[0] + r2[1] * t2[1] + r2[2] * t2[2];
    const double det = a * e - b * c;
    tref[t] = e / det;
    tref[ts + t] = -b / det;
    tref[2 * ts + t] = -c / det;
    tref[3 * ts + t] = a / det;
    tref[4 * ts + t] = 0.5 * sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
}

// Inside (1) / outside (0) of every cell of droplet d from the crossing
// tables, one lane per cell.
__global__ __launch_bounds__(kBlock) void k_inside_mask(const DropDev* __restrict__ drops, int d,
                                                        const int* __restrict__ cnt,
                                                        const double* __restrict__ xs,
                                                        uint8_t* __restrict__ mask) {
    const DropDev& D = drops[d];
    const int cell = blockIdx.x * kBlock + threadIdx.x;
    if (cell >= D.ncell) return;
    const int x = cell % D.nx, row = cell / D.nx;
    mask[cell] = cell_inside(D, cnt, xs, x, row) ? 1 : 0;
}

// ---------------------------------------------------------------------------
// Interpolation (eq. vel_interpolation) + forward-Euler advection
// ---------------------------------------------------------------------------
template <int DIM, bool ONE>
__global__ __launch_bounds__(kNodeBlock) void k_interp_advect(const DropDev* __restrict__ drops,
                                                          NodeArrays A,
                                                          const float* __restrict__ U_all,
                                                          int* __restrict__ status) {
    // G lanes per node, each taking T / G taps (k, k + G, ...)
    constexpr int T = Taps<DIM>::n, G = InterpLanes<DIM>::n, R = T / G;
    const int gid = blockIdx.x * kNodeBlock + threadIdx.x;
    const int j = gid / G, k = gid % G;
    if (j >= A.ntot) return;
    const int d = node_droplet<ONE>(A, j);
    const DropDev& D = drops[d];
    const int st = A.stride;
    if (!D.active || D.force_mode != 0) {
        hold_position<DIM>(A, j, k);
        return;
    }
    double q[3] = {0, 0, 0};
    bool ok = true;
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        q[a] = A.pos[a * st + j];
        ok = ok && coord_ok(q[a]);
    }
    if (!ok) {
        hold_position<DIM>(A, j, k);
        if (k == 0) atomicOr(status + d, 4);
        return;
    }
    const float* __restrict__ U = U_all + (long long)DIM * D.c_off;
    float w[R];
    int cell[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        int row, ix;
        cell[r] = lane_tap<DIM>(D, q, k + r * G, w[r], row, ix);
    }
    // every gather is issued before any is used: a tap beyond a wall, where
    // the fluid is at rest, reads cell 0 with weight zero
    float u[R][3];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int c = cell[r] >= 0 ? cell[r] : 0;
#pragma unroll
        for (int a = 0; a < DIM; ++a) u[r][a] = U[a * D.ncell + c];
    }
    float acc[3] = {0.f, 0.f, 0.f};
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const float wr = cell[r] >= 0 ? w[r] : 0.f;
#pragma unroll
        for (int a = 0; a < DIM; ++a) acc[a] += u[r][a] * wr;
    }
#pragma unroll
    for (int a = 0; a < DIM; ++a) acc[a] = group_sum<G>(acc[a]);
    if (k != 0) return;
    double dq[2] = {0.0, 0.0};
    if (DIM == 2 && D.respace != 0.0) {
        int jm, jp;
        ring_2d(D, j, jm, jp);
        const double qm[3] = {A.pos[jm], A.pos[st + jm], 0.0}, qp[3] = {A.pos[jp], A.pos[st + jp], 0.0};
        if (!(coord_ok(qm[0]) && coord_ok(qm[1]) && coord_ok(qp[0]) && coord_ok(qp[1]))) {
#pragma unroll
            for (int a = 0; a < DIM; ++a) hold_position<DIM>(A, j, a);
            atomicOr(status + d, 4);
            return;
        }
        respace_move(D.respace, qm, q, qp, dq);
    }
    float sp = 0.f;
    double qn[DIM];
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        qn[a] = (q[a] + (double)acc[a]) + (a < 2 ? dq[a] : 0.0);
        A.qdot[a * st + j] = acc[a];
        A.pos_w[a * st + j] = qn[a];
        sp += acc[a] * acc[a];
    }
    int bad = 0;
    if (!(sp <= 0.09f)) bad |= 2;  // |qdot| > 0.3 or not finite
    if (D.wetting && !(qn[DIM - 1] > 0.0)) bad |= 1;
    if (bad) atomicOr(status + d, bad);
}

// ---------------------------------------------------------------------------
// 3D: nodal forces, then spreading aggregated in LDS (eq. force_spread)
// ---------------------------------------------------------------------------
template <int G>
__device__ __forceinline__ double group_sum_d(double v) {
#pragma unroll
    for (int o = G / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Forces of every vertex (membrane + wetting): a group of kForceLanes lanes
// per vertex, each lane taking its own incident triangles (one for the
// usual vertex), their contributions summed across the group; the group's
// first lane adds the wetting term and writes the force.  Against one lane
// per vertex that walks its triangles in turn (three batched rounds of
// loads, then 5-6 FP64 triangle evaluations in sequence) the chain per lane
// is one triangle long and the launch has eight times the wavefronts.
constexpr int kForceLanes = 8;
template <bool ONE>
__global__ __launch_bounds__(kBlock) void k_force3(const DropDev* __restrict__ drops, NodeArrays A) {
    const int gid = blockIdx.x * kBlock + threadIdx.x;
    const int j = gid / kForceLanes, k = gid % kForceLanes;
    if (j >= A.ntot) return;  // the whole group leaves together
    const DropDev& D = drops[node_droplet<ONE>(A, j)];
    if (!D.active || D.force_mode != 0) return;
    const int st = A.stride, ts = A.tstride;
    const double q[3] = {A.pos[j], A.pos[st + j], A.pos[2 * st + j]};
    const int beg = A.inc_beg[j], cnt = A.inc_end[j] - beg;
    double fs[3] = {0.0, 0.0, 0.0}, ns[3] = {0.0, 0.0, 0.0}, chi = 0.0;
    for (int i = k; i < cnt; i += kForceLanes) {
        const int e = A.inc[beg + i];
        const int t = e >> 2, s = e & 3;
        const int sb = s == 2 ? 0 : s + 1, sc = s == 0 ? 2 : s - 1;
        const int vb = A.tri[sb * ts + t], vc = A.tri[sc * ts + t];
        // vertex slot s of triangle t is node j itself
        double P[3][3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            P[s][a] = q[a];
            P[sb][a] = A.pos[a * st + vb];
            P[sc][a] = A.pos[a * st + vc];
        }
        tri_contrib(D, A, t, s, P, fs, ns, chi);
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        fs[a] = group_sum_d<kForceLanes>(fs[a]);
        ns[a] = group_sum_d<kForceLanes>(ns[a]);
    }
    chi = group_sum_d<kForceLanes>(chi);
    if (k != 0) return;
    if (D.wetting) {
        const double nn = sqrt(ns[0] * ns[0] + ns[1] * ns[1] + ns[2] * ns[2]);
        const double P = wetting_pi(D, q[2]);
#pragma unroll
        for (int a = 0; a < 3; ++a) fs[a] -= (chi / 3.0) * P * (ns[a] / nn);
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) A.phi[a * A.stride + j] = (float)fs[a];
}

// A workgroup spreads one chunk of up to kChunk vertices that are close in
// space (consecutive in Morton order, cut by the host where the taps' box
// would grow beyond a budget).  Their 64 taps each overlap heavily,
// so the contributions are first summed in an LDS box that covers the
// chunk's taps, and each touched cell then takes one global atomic add per
// component instead of one per contribution.  A chunk whose box exceeds
// kBoxCells (vertices far apart) adds straight to global memory.
// Chunks of 16 vertices, 256-lane workgroups and a 1024-cell box measured
// fastest among chunks of 8-64 vertices and 128-1024 lanes (3D steps of
// 256x256x128 and 240x240x130: 295 and 348 us against 312 and 374 us for
// 64 vertices on 1024 lanes), and again with the 64-bit fixed-point sums
// (256x256x128 step 271 us against 273-278 us for chunks of 8-32 vertices,
// 128-512 lanes and boxes of 512-2048 cells).
#ifndef IBLB_SPREAD_CHUNK
#define IBLB_SPREAD_CHUNK 16
#endif
#ifndef IBLB_SPREAD_BOX
#define IBLB_SPREAD_BOX 1024
#endif
#ifndef IBLB_SPREAD_BLOCK
#define IBLB_SPREAD_BLOCK 256
#endif
constexpr int kChunk = IBLB_SPREAD_CHUNK;
constexpr int kBoxCells = IBLB_SPREAD_BOX;
constexpr int kSpreadBlock = IBLB_SPREAD_BLOCK;  // wavefronts each taking every (block / 64)-th vertex

__global__ __launch_bounds__(kSpreadBlock) void k_spread3(const DropDev* __restrict__ drops, NodeArrays A,
                                                    const int4* __restrict__ chunks,
                                                    unsigned long long* __restrict__ Fq_all,
                                                    uint8_t* __restrict__ flags_all,
                                                    int* __restrict__ status, int want_dropped) {
    __shared__ unsigned long long box[3 * kBoxCells];
    __shared__ uint8_t touched[kBoxCells];
    __shared__ double sq[kChunk][3];
    __shared__ float sph[kChunk][3];
    __shared__ int sok[kChunk];
    __shared__ int lo[3], hi[3];
    const int4 ch = chunks[blockIdx.x];  // (droplet, first index into perm, count, -)
    const int t = threadIdx.x, st = A.stride, count = ch.z;
    // the chunk's vertices (positions and forces together) are fetched
    // before the droplet's parameters are checked, not after them
    double q[3] = {0.0, 0.0, 0.0};
    float ph[3] = {0.f, 0.f, 0.f};
    if (t < count) {
        const int j = A.perm[ch.y + t];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            q[a] = A.pos[a * st + j];
            ph[a] = A.phi[a * st + j];
        }
    }
    const DropDev& D = drops[ch.x];
    if (!D.active || D.force_mode != 0) return;
    if (t < 3) {
        lo[t] = INT_MAX;
        hi[t] = INT_MIN;
    }
    __syncthreads();
    if (t < count) {
        bool ok = true;
#pragma unroll
        for (int a = 0; a < 3; ++a) ok = ok && coord_ok(q[a]);
        sok[t] = ok;
        if (ok) {
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                sq[t][a] = q[a];
                sph[t][a] = ph[a];
                const int b = (int)floor(q[a] - 0.5) - 1;
                atomicMin(&lo[a], b);
                atomicMax(&hi[a], b);
            }
        } else {
            atomicOr(status + ch.x, 4);
        }
    }
    __syncthreads();
    const int ex = hi[0] - lo[0] + 4, ey = hi[1] - lo[1] + 4, ez = hi[2] - lo[2] + 4;
    const bool any = lo[0] <= hi[0];
    const bool fits = any && (long long)ex * ey * ez <= kBoxCells;
    const int ncb = fits ? ex * ey * ez : 0;
    for (int c = t; c < ncb; c += kSpreadBlock) {
        box[c] = 0;
        box[kBoxCells + c] = 0;
        box[2 * kBoxCells + c] = 0;
        touched[c] = 0;
    }
    __syncthreads();
    unsigned long long* __restrict__ Fq = Fq_all + 3LL * D.c_off;
    bool fine = true;
    const int k = t & 63;  // tap of this lane; one vertex per wavefront at a time
    const int kx = k & 3, ky = (k >> 2) & 3, kz = k >> 4;
    for (int v = t >> 6; v < count; v += kSpreadBlock / 64) {
        if (!sok[v]) continue;  // the same for the whole wavefront
        int bx, by, bz;
        const float w = peskin_tap(sq[v][0], kx, bx) * peskin_tap(sq[v][1], ky, by) *
                        peskin_tap(sq[v][2], kz, bz);
        const int gx = tap_index(bx, kx, D.nx, D.bcx), gy = tap_index(by, ky, D.ny, D.bcy),
                  gz = tap_index(bz, kz, D.nz, D.bcz);
        float lost[3] = {0.f, 0.f, 0.f};
        if ((gx | gy | gz) < 0) {
#pragma unroll
            for (int a = 0; a < 3; ++a) lost[a] = sph[v][a] * w;
        } else if (fits) {
            const int c = ((bz + kz - lo[2]) * ey + (by + ky - lo[1])) * ex + (bx + kx - lo[0]);
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const float val = sph[v][a] * w;
                if (fq_ok(val))
                    atomicAdd(&box[a * kBoxCells + c], fq_of(val));
                else
                    fine = false;
            }
            touched[c] = 1;
        } else {
            const int row = gz * D.ny + gy, cell = row * D.nx + gx;
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const float val = sph[v][a] * w;
                if (fq_ok(val))
                    atomicAdd(Fq + a * D.ncell + cell, fq_of(val));
                else
                    fine = false;
            }
            flags_all[D.flag_off + row * D.nstrip + (gx >> D.sshift)] = 1;
        }
        if (want_dropped) {
#pragma unroll
            for (int a = 0; a < 3; ++a) lost[a] = group_sum<64>(lost[a]);
            if (k == 0) {
                const int j = A.perm[ch.y + v];
#pragma unroll
                for (int a = 0; a < 3; ++a) A.dropped[a * st + j] = lost[a];
            }
        }
    }
    if (!fine) atomicOr(status + ch.x, 2);
    if (!fits) return;
    __syncthreads();
    for (int c = t; c < ncb; c += kSpreadBlock) {
        if (!touched[c]) continue;
        const int cx = c % ex, cy = (c / ex) % ey, cz = c / (ex * ey);
        // a touched cell received a fluid tap, so none of these is -1
        const int gx = tap_index(lo[0], cx, D.nx, D.bcx), gy = tap_index(lo[1], cy, D.ny, D.bcy),
                  gz = tap_index(lo[2], cz, D.nz, D.bcz);
        const int row = gz * D.ny + gy, cell = row * D.nx + gx;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const unsigned long long v = box[a * kBoxCells + c];
            if (v != 0) atomicAdd(Fq + a * D.ncell + cell, v);
        }
        flags_all[D.flag_off + row * D.nstrip + (gx >> D.sshift)] = 1;
    }
}

// ---------------------------------------------------------------------------
// 2D: interpolation + advection of step t fused with the forces and the
// spreading of step t + 1
// ---------------------------------------------------------------------------
// The lanes of node j's group also interpolate at its two ring neighbours,
// so the new positions that the force at j needs are formed in registers
// and no grid-wide wait separates the two halves.  Reads positions A.pos
// (step t), writes A.pos_w (step t + 1).
template <bool ONE>
__global__ __launch_bounds__(kNodeBlock) void k_ib_fused2(const DropDev* __restrict__ drops, NodeArrays A,
                                                      const float* __restrict__ U_all,
                                                      unsigned long long* __restrict__ Fq_all,
                                                      uint8_t* __restrict__ flags_all,
                                                      int* __restrict__ status, int want_dropped,
                                                      int* __restrict__ xcnt,
                                                      double* __restrict__ xpos) {
    constexpr int T = Taps<2>::n;
    const int gid = blockIdx.x * kNodeBlock + threadIdx.x;
    const int j = gid / T, k = gid % T;
    if (j >= A.ntot) return;
    const int d = node_droplet<ONE>(A, j);
    const int st = A.stride;
    // a lone droplet's ring is nodes 0 .. ntot - 1, so its positions are
    // fetched alongside the droplet's parameters instead of after them
    int jm = 0, jp = 0;
    double q[3][3];
    if constexpr (ONE) {
        jm = j == 0 ? A.ntot - 1 : j - 1;
        jp = j == A.ntot - 1 ? 0 : j + 1;
        const int id[3] = {jm, j, jp};
#pragma unroll
        for (int m = 0; m < 3; ++m) {
            q[m][0] = A.pos[id[m]];
            q[m][1] = A.pos[st + id[m]];
        }
    }
    const DropDev& D = drops[d];
    if (!D.active || D.force_mode != 0) {
        hold_position<2>(A, j, k);
        return;
    }
    if constexpr (!ONE) {
        ring_2d(D, j, jm, jp);
        const int id[3] = {jm, j, jp};
#pragma unroll
        for (int m = 0; m < 3; ++m) {
            q[m][0] = A.pos[id[m]];
            q[m][1] = A.pos[st + id[m]];
        }
    }
    // with re-spacing, the ring neighbours' moves need their own outer
    // neighbours: qo[0] before jm, qo[1] after jp
    const bool resp = D.respace != 0.0;
    double qo[2][3] = {{0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}};
    if (resp) {
        int jmm, jpp, dummy;
        ring_2d(D, jm, jmm, dummy);
        ring_2d(D, jp, dummy, jpp);
        qo[0][0] = A.pos[jmm];
        qo[0][1] = A.pos[st + jmm];
        qo[1][0] = A.pos[jpp];
        qo[1][1] = A.pos[st + jpp];
    }
    bool ok = !resp || (coord_ok(qo[0][0]) && coord_ok(qo[0][1]) && coord_ok(qo[1][0]) && coord_ok(qo[1][1]));
#pragma unroll
    for (int m = 0; m < 3; ++m) {
        q[m][2] = 0.0;
        ok = ok && coord_ok(q[m][0]) && coord_ok(q[m][1]);
    }
    if (!ok) {
        hold_position<2>(A, j, k);
        if (k == 0) atomicOr(status + d, 4);
        return;
    }
    const float* __restrict__ U = U_all + 2LL * D.c_off;
    float w[3];
    int cell[3];
#pragma unroll
    for (int m = 0; m < 3; ++m) {
        int row, ix;
        cell[m] = lane_tap<2>(D, q[m], k, w[m], row, ix);
    }
    // all six gathers are issued before any is used (a conditional load per
    // tap would wait for each in turn): a tap beyond a wall, where the fluid
    // is at rest, reads cell 0 with weight zero
    float u[3][2];
#pragma unroll
    for (int m = 0; m < 3; ++m) {
        const int c = cell[m] >= 0 ? cell[m] : 0;
        u[m][0] = U[c];
        u[m][1] = U[D.ncell + c];
    }
    float acc[3][2];
#pragma unroll
    for (int m = 0; m < 3; ++m) {
        const float wm = cell[m] >= 0 ? w[m] : 0.f;
        acc[m][0] = u[m][0] * wm;
        acc[m][1] = u[m][1] * wm;
    }
#pragma unroll
    for (int m = 0; m < 3; ++m) {
        acc[m][0] = group_sum<T>(acc[m][0]);
        acc[m][1] = group_sum<T>(acc[m][1]);
    }
    double qn[3][3];
#pragma unroll
    for (int m = 0; m < 3; ++m) {
        qn[m][0] = q[m][0] + (double)acc[m][0];
        qn[m][1] = q[m][1] + (double)acc[m][1];
        qn[m][2] = 0.0;
    }
    if (resp) {
        double dq[2];
        respace_move(D.respace, qo[0], q[0], q[1], dq);
        qn[0][0] += dq[0];
        qn[0][1] += dq[1];
        respace_move(D.respace, q[0], q[1], q[2], dq);
        qn[1][0] += dq[0];
        qn[1][1] += dq[1];
        respace_move(D.respace, q[1], q[2], qo[1], dq);
        qn[2][0] += dq[0];
        qn[2][1] += dq[1];
    }
    if (k == 0) {
        A.qdot[j] = acc[1][0];
        A.qdot[st + j] = acc[1][1];
        A.pos_w[j] = qn[1][0];
        A.pos_w[st + j] = qn[1][1];
        int bad = 0;
        if (!(acc[1][0] * acc[1][0] + acc[1][1] * acc[1][1] <= 0.09f)) bad |= 2;
        if (D.wetting && !(qn[1][1] > 0.0)) bad |= 1;
        if (bad) atomicOr(status + d, bad);
    }
    ok = true;
#pragma unroll
    for (int m = 0; m < 3; ++m) ok = ok && coord_ok(qn[m][0]) && coord_ok(qn[m][1]);
    if (!ok) {
        if (k == 0) atomicOr(status + d, 4);
        return;
    }
    // crossings of edge j -> j+1 at the new positions, for the next step
    if (D.visc && k == 1) cross_edge_2d(D, xcnt, xpos, qn[1], qn[2], status, d);
    double fs[2], n[2], chi;
    geom_2d(D.sigma, qn[0], qn[1], qn[2], fs, n, chi);
    if (D.wetting) {
        const double P = wetting_pi(D, qn[1][1]);
        fs[0] -= 0.5 * chi * P * n[0];
        fs[1] -= 0.5 * chi * P * n[1];
    }
    const float ph[3] = {(float)fs[0], (float)fs[1], 0.f};
    if (k == 0) {
        A.phi[j] = ph[0];
        A.phi[st + j] = ph[1];
    }
    spread_lane<2>(D, A, j, k, qn[1], ph, Fq_all, flags_all, want_dropped, status + d);
}

// ---------------------------------------------------------------------------
// Population I/O and initialisation
// ---------------------------------------------------------------------------
// Equilibrium populations (eq. f^eq, deviation form f_eq - w =
// w (rho - 1) + w rho (3 c.u + 4.5 (c.u)^2 - 1.5 u^2)) from a density field
// (null: 1) and a velocity field [dim][ncell] (null: 0), one lane per cell.
// nxy cells per plane of the fields, ppl elements per plane of the
// population arrays.
__device__ __forceinline__ int pop_cell(int cell, int nxy, int ppl) { return cell + cell / nxy * (ppl - nxy); }

template <int DIM, int S>
__global__ void k_init_eq(typename Codec<S>::T* __restrict__ f, int ncell, int fst, int nxy, int ppl,
                          const float* __restrict__ rho_in, const float* __restrict__ u_in) {
    using L = Lattice<DIM>;
    const int cell = blockIdx.x * kBlock + threadIdx.x;
    if (cell >= ncell) return;
    const int pc = pop_cell(cell, nxy, ppl);
    const float rho = rho_in ? rho_in[cell] : 1.f;
    float u[3] = {0.f, 0.f, 0.f};
    if (u_in)
#pragma unroll
        for (int a = 0; a < DIM; ++a) u[a] = u_in[a * ncell + cell];
    const float usq = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
#pragma unroll
    for (int i = 0; i < L::Q; ++i) {
        const float cu = L::c[i][0] * u[0] + L::c[i][1] * u[1] + (DIM == 3 ? L::c[i][2] * u[2] : 0.f);
        const float v = L::w[i] * ((rho - 1.f) + rho * (3.f * cu + 4.5f * cu * cu - 1.5f * usq));
        Codec<S>::store(f, i * fst + pc, v);
    }
}

// Dense [Q][ncell] doubles on the caller's side, population arrays fst
// elements apart in the workspace, their planes ppl elements apart.
template <int S>
__global__ void k_pop_write(typename Codec<S>::T* __restrict__ f, int ncell, int fst, int nxy, int ppl,
                            long long n, const double* __restrict__ src) {
    const long long i = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) f[(i / ncell) * fst + pop_cell((int)(i % ncell), nxy, ppl)] = Codec<S>::from_double(src[i]);
}

template <int S>
__global__ void k_pop_read(const typename Codec<S>::T* __restrict__ f, int ncell, int fst, int nxy, int ppl,
                           long long n, double* __restrict__ dst) {
    const long long i = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) dst[i] = Codec<S>::to_double(f[(i / ncell) * fst + pop_cell((int)(i % ncell), nxy, ppl)]);
}

// Streaming copy used to measure the attainable HBM bandwidth of the device:
// each lane moves four 16-byte vectors, all loads issued before the stores.
typedef float v4f __attribute__((ext_vector_type(4)));

template <int NT>
__global__ __launch_bounds__(kBlock) void k_copy_probe(const v4f* __restrict__ src,
                                                       v4f* __restrict__ dst, long long n) {
    const long long base = (long long)blockIdx.x * (4 * kBlock) + threadIdx.x;
    v4f v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const long long i = base + (long long)u * kBlock;
        if (i < n) v[u] = NT ? __builtin_nontemporal_load(src + i) : src[i];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const long long i = base + (long long)u * kBlock;
        if (i < n) {
            if (NT)
                __builtin_nontemporal_store(v[u], dst + i);
            else
                dst[i] = v[u];
        }
    }
}

__global__ void k_fill_f32(float* __restrict__ p, long long n, float v) {
    const long long i = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) p[i] = v;
}

// ---------------------------------------------------------------------------
// Diagnostics
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
template <typename T>
__device__ __forceinline__ T wave_min(T v) {
    for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
    return v;
}
template <typename T>
__device__ __forceinline__ T wave_max(T v) {
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

// Block-wide reduction of 256 threads (4 wavefronts); every thread gets the
// result.  kind: 0 sum, 1 min, 2 max.
__device__ double block_reduce(double v, int kind, double* sh) {
    v = kind == 0 ? wave_sum(v) : (kind == 1 ? wave_min(v) : wave_max(v));
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sh[w] = v;
    __syncthreads();
    double r = sh[0];
    for (int k = 1; k < kBlock / 64; ++k)
        r = kind == 0 ? r + sh[k] : (kind == 1 ? fmin(r, sh[k]) : fmax(r, sh[k]));
    return r;
}

// Per-tile partial sums over cells: [0] sum of f - w, [1..3] rho U,
// [4..6] F of the last step.
template <int DIM, int S, int BX>
__global__ __launch_bounds__(kBlock) void k_cell_sums(const DropDev* __restrict__ drops,
                                                      const int4* __restrict__ tiles,
                                                      const typename Codec<S>::T* __restrict__ f_all,
                                                      const float* __restrict__ U_all,
                                                      const float* __restrict__ rho_all,
                                                      const float* __restrict__ Fout_all,
                                                      double* __restrict__ partials) {
    __shared__ double sh[kBlock / 64];
    using L = Lattice<DIM>;
    constexpr int BY = kBlock / BX;
    const int t = blockIdx.x;
    const int4 tile = tiles[t];
    const DropDev& D = drops[tile.x];
    const int x = tile.y * BX + (int)(threadIdx.x % BX);
    const int y = tile.z * BY + (int)(threadIdx.x / BX);
    const int z = tile.w;
    double v[7] = {0, 0, 0, 0, 0, 0, 0};
    if (x < D.nx && y < D.ny) {
        const int ncell = D.ncell;
        const int cell = (z * D.ny + y) * D.nx + x;
        const typename Codec<S>::T* f = f_all + D.f_off;
        double s = 0.0;
        const int pc = z * D.ppl + y * D.nx + x;
        for (int i = 0; i < L::Q; ++i) s += (double)Codec<S>::load(f, i * D.fst + pc);
        v[0] = s;
        const double rho = rho_all[D.c_off + cell];
        const float* U = U_all + (long long)DIM * D.c_off;
        const float* Fo = Fout_all + (long long)DIM * D.c_off;
        for (int a = 0; a < DIM; ++a) {
            v[1 + a] = rho * (double)U[a * ncell + cell];
            v[4 + a] = (double)Fo[a * ncell + cell];
        }
    }
    for (int k = 0; k < 7; ++k) {
        const double r = block_reduce(v[k], 0, sh);
        if (threadIdx.x == 0) partials[(long long)t * 8 + k] = r;
    }
}

// One block per droplet: cell partials + interface reductions.
// partials may be null: interface quantities only (cell sums left zero).
template <int DIM>
__global__ __launch_bounds__(kBlock) void k_diag(const DropDev* __restrict__ drops, NodeArrays A,
                                                 const double* __restrict__ partials,
                                                 DiagDev* __restrict__ out) {
    __shared__ double sh[kBlock / 64];
    const int d = blockIdx.x;
    const DropDev& D = drops[d];
    DiagDev r;
    double acc[7] = {0, 0, 0, 0, 0, 0, 0};
    if (partials)
        for (int t = D.tile_off + threadIdx.x; t < D.tile_off + D.n_tiles; t += kBlock)
            for (int k = 0; k < 7; ++k) acc[k] += partials[(long long)t * 8 + k];
    for (int k = 0; k < 7; ++k) acc[k] = block_reduce(acc[k], 0, sh);
    r.mass_dev = acc[0];
    for (int a = 0; a < 3; ++a) {
        r.mom[a] = acc[1 + a];
        r.sum_F[a] = acc[4 + a];
    }

    const int st = A.stride, N = D.n_nodes, j0 = D.node_off;
    double sphi[3] = {0, 0, 0}, sdrop[3] = {0, 0, 0};
    double vol = 0, area = 0, hmin = 1e300, hmax = -1e300, un = 0, us = 0;
    double emin = 1e300, emax = 0, lo = 1e300, hi = -1e300, cx = 0, cy = 0, cn = 0;
    const double zc = D.zcut;
    for (int l = threadIdx.x; l < N; l += kBlock) {
        const int j = j0 + l;
        double q[3], fs[3], n[3], chi;
        if (DIM == 2) {
            node_geom_2d(D, A, j, q, fs, n, chi);
        } else {
            node_geom_3d(D, A, j, q, fs, n, chi);
        }
        double u2 = 0, udn = 0;
        for (int a = 0; a < DIM; ++a) {
            sphi[a] += A.phi[a * st + j];
            sdrop[a] += A.dropped[a * st + j];
            const double v = A.qdot[a * st + j];
            u2 += v * v;
            udn += v * n[a];
        }
        un = fmax(un, fabs(udn));
        us = fmax(us, sqrt(u2));
        hmin = fmin(hmin, q[DIM - 1]);
        hmax = fmax(hmax, q[DIM - 1]);
        if (DIM == 2) {
            const int jp = j0 + (l == N - 1 ? 0 : l + 1);
            const double x0 = q[0], y0 = q[1], x1 = A.pos[jp], y1 = A.pos[st + jp];
            vol += 0.5 * (x0 * y1 - x1 * y0);
            const double e = sqrt((x1 - x0) * (x1 - x0) + (y1 - y0) * (y1 - y0));
            area += e;
            emin = fmin(emin, e);
            emax = fmax(emax, e);
            const double a0 = y0 - zc, a1 = y1 - zc;
            if (a0 * a1 < 0.0 || (a0 == 0.0 && a1 != 0.0)) {
                const double xs = x0 + a0 / (a0 - a1) * (x1 - x0);
                lo = fmin(lo, xs);
                hi = fmax(hi, xs);
            }
        }
    }
    if (DIM == 3) {
        const int ts = A.tstride;
        for (int t = D.tri_off + threadIdx.x; t < D.tri_off + D.n_tris; t += kBlock) {
            const int v[3] = {A.tri[t], A.tri[ts + t], A.tri[2 * ts + t]};
            double P[3][3];
            for (int m = 0; m < 3; ++m)
                for (int a = 0; a < 3; ++a) P[m][a] = A.pos[a * st + v[m]];
            const double cr[3] = {P[1][1] * P[2][2] - P[1][2] * P[2][1],
                                  P[1][2] * P[2][0] - P[1][0] * P[2][2],
                                  P[1][0] * P[2][1] - P[1][1] * P[2][0]};
            vol += (P[0][0] * cr[0] + P[0][1] * cr[1] + P[0][2] * cr[2]) / 6.0;
            const double e1[3] = {P[1][0] - P[0][0], P[1][1] - P[0][1], P[1][2] - P[0][2]};
            const double e2[3] = {P[2][0] - P[0][0], P[2][1] - P[0][1], P[2][2] - P[0][2]};
            const double nt[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2],
                                  e1[0] * e2[1] - e1[1] * e2[0]};
            area += 0.5 * sqrt(nt[0] * nt[0] + nt[1] * nt[1] + nt[2] * nt[2]);
            for (int m = 0; m < 3; ++m) {
                const int m1 = m == 2 ? 0 : m + 1;
                const double dx = P[m1][0] - P[m][0], dy = P[m1][1] - P[m][1],
                             dz = P[m1][2] - P[m][2];
                const double e = sqrt(dx * dx + dy * dy + dz * dz);
                emin = fmin(emin, e);
                emax = fmax(emax, e);
                if (v[m] < v[m1]) {  // each edge once
                    const double a0 = P[m][2] - zc, a1 = P[m1][2] - zc;
                    if (a0 * a1 < 0.0) {
                        const double s = a0 / (a0 - a1);
                        cx += P[m][0] + s * dx;
                        cy += P[m][1] + s * dy;
                        cn += 1.0;
                    }
                }
            }
        }
    }
    for (int a = 0; a < 3; ++a) {
        r.sum_phi[a] = block_reduce(sphi[a], 0, sh);
        r.dropped[a] = block_reduce(sdrop[a], 0, sh);
    }
    r.volume = block_reduce(vol, 0, sh);
    r.area = block_reduce(area, 0, sh);
    r.min_h = block_reduce(hmin, 1, sh);
    r.max_h = block_reduce(hmax, 2, sh);
    r.max_un = block_reduce(un, 2, sh);
    r.max_u = block_reduce(us, 2, sh);
    r.edge_min = block_reduce(emin, 1, sh);
    r.edge_max = block_reduce(emax, 2, sh);
    r.cross_lo = block_reduce(lo, 1, sh);
    r.cross_hi = block_reduce(hi, 2, sh);
    r.cross_r = 0.0;
    r.cross_n = 0.0;
    if (DIM == 3) {
        const double n = block_reduce(cn, 0, sh);
        const double mx = block_reduce(cx, 0, sh) / n, my = block_reduce(cy, 0, sh) / n;
        double dsum = 0.0;
        const int ts = A.tstride;
        for (int t = D.tri_off + threadIdx.x; t < D.tri_off + D.n_tris; t += kBlock) {
            const int v[3] = {A.tri[t], A.tri[ts + t], A.tri[2 * ts + t]};
            for (int m = 0; m < 3; ++m) {
                const int m1 = m == 2 ? 0 : m + 1;
                if (v[m] >= v[m1]) continue;
                const double z0 = A.pos[2 * st + v[m]] - zc, z1 = A.pos[2 * st + v[m1]] - zc;
                if (z0 * z1 < 0.0) {
                    const double s = z0 / (z0 - z1);
                    const double px = A.pos[v[m]] + s * (A.pos[v[m1]] - A.pos[v[m]]);
                    const double py = A.pos[st + v[m]] + s * (A.pos[st + v[m1]] - A.pos[st + v[m]]);
                    dsum += sqrt((px - mx) * (px - mx) + (py - my) * (py - my));
                }
            }
        }
        r.cross_r = block_reduce(dsum, 0, sh) / n;
        r.cross_n = n;
    }
    if (threadIdx.x == 0) out[d] = r;
}

// Contact radius of droplet d at the positions A.pos by the two protocols
// of Sec. Dynamics, one workgroup.  (i) the interface cut by the plane
// (2D: line) at height zcut: 2D half the distance between the outermost
// crossings, 3D the mean distance of the edge crossings to their centre.
// (ii) the flat lower region: the elements (2D edges, 3D triangles) whose
// nodes all lie below the mid-height between the lowest and the highest
// node and differ in height by less than tol; 2D half its length, 3D the
// radius of the disc of its area.  out: r_i (NaN without crossings), r_ii,
// number of crossings.
template <int DIM>
__global__ __launch_bounds__(kBlock) void k_contact(const DropDev* __restrict__ drops, int d, NodeArrays A,
                                                    double zcut, double tol, double* __restrict__ out) {
    __shared__ double sh[kBlock / 64];
    const DropDev& D = drops[d];
    const int st = A.stride, N = D.n_nodes, j0 = D.node_off, H = DIM - 1;
    double hmin = 1e300, hmax = -1e300;
    for (int l = threadIdx.x; l < N; l += kBlock) {
        const double h = A.pos[H * st + j0 + l];
        hmin = fmin(hmin, h);
        hmax = fmax(hmax, h);
    }
    hmin = block_reduce(hmin, 1, sh);
    hmax = block_reduce(hmax, 2, sh);
    const double mid = 0.5 * (hmin + hmax);
    double lo = 1e300, hi = -1e300, cx = 0.0, cy = 0.0, cn = 0.0, flat = 0.0;
    const int ts = A.tstride;
    if (DIM == 2) {
        for (int l = threadIdx.x; l < N; l += kBlock) {
            const int j = j0 + l, jp = j0 + (l == N - 1 ? 0 : l + 1);
            const double x0 = A.pos[j], y0 = A.pos[st + j], x1 = A.pos[jp], y1 = A.pos[st + jp];
            const double a0 = y0 - zcut, a1 = y1 - zcut;
            if (a0 * a1 < 0.0 || (a0 == 0.0 && a1 != 0.0)) {
                const double xs = x0 + a0 / (a0 - a1) * (x1 - x0);
                lo = fmin(lo, xs);
                hi = fmax(hi, xs);
                cn += 1.0;
            }
            if (y0 < mid && y1 < mid && fabs(y1 - y0) < tol)
                flat += sqrt((x1 - x0) * (x1 - x0) + (y1 - y0) * (y1 - y0));
        }
    } else {
        for (int t = D.tri_off + threadIdx.x; t < D.tri_off + D.n_tris; t += kBlock) {
            const int v[3] = {A.tri[t], A.tri[ts + t], A.tri[2 * ts + t]};
            double P[3][3];
            for (int m = 0; m < 3; ++m)
                for (int a = 0; a < 3; ++a) P[m][a] = A.pos[a * st + v[m]];
            for (int m = 0; m < 3; ++m) {
                const int m1 = m == 2 ? 0 : m + 1;
                if (v[m] >= v[m1]) continue;  // each edge once
                const double a0 = P[m][2] - zcut, a1 = P[m1][2] - zcut;
                if (a0 * a1 < 0.0) {
                    const double s = a0 / (a0 - a1);
                    cx += P[m][0] + s * (P[m1][0] - P[m][0]);
                    cy += P[m][1] + s * (P[m1][1] - P[m][1]);
                    cn += 1.0;
                }
            }
            const double zlo = fmin(fmin(P[0][2], P[1][2]), P[2][2]);
            const double zhi = fmax(fmax(P[0][2], P[1][2]), P[2][2]);
            if (zhi < mid && zhi - zlo < tol) {
                const double e1[3] = {P[1][0] - P[0][0], P[1][1] - P[0][1], P[1][2] - P[0][2]};
                const double e2[3] = {P[2][0] - P[0][0], P[2][1] - P[0][1], P[2][2] - P[0][2]};
                const double nt[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2],
                                      e1[0] * e2[1] - e1[1] * e2[0]};
                flat += 0.5 * sqrt(nt[0] * nt[0] + nt[1] * nt[1] + nt[2] * nt[2]);
            }
        }
    }
    lo = block_reduce(lo, 1, sh);
    hi = block_reduce(hi, 2, sh);
    cn = block_reduce(cn, 0, sh);
    flat = block_reduce(flat, 0, sh);
    double ri = __builtin_nan("");
    if (DIM == 2) {
        if (cn >= 2.0) ri = 0.5 * (hi - lo);
    } else {
        cx = block_reduce(cx, 0, sh);
        cy = block_reduce(cy, 0, sh);
        double dsum = 0.0;
        if (cn > 0.0) {
            const double mx = cx / cn, my = cy / cn;
            for (int t = D.tri_off + threadIdx.x; t < D.tri_off + D.n_tris; t += kBlock) {
                const int v[3] = {A.tri[t], A.tri[ts + t], A.tri[2 * ts + t]};
                for (int m = 0; m < 3; ++m) {
                    const int m1 = m == 2 ? 0 : m + 1;
                    if (v[m] >= v[m1]) continue;
                    const double z0 = A.pos[2 * st + v[m]] - zcut, z1 = A.pos[2 * st + v[m1]] - zcut;
                    if (z0 * z1 < 0.0) {
                        const double s = z0 / (z0 - z1);
                        const double px = A.pos[v[m]] + s * (A.pos[v[m1]] - A.pos[v[m]]);
                        const double py = A.pos[st + v[m]] + s * (A.pos[st + v[m1]] - A.pos[st + v[m]]);
                        dsum += sqrt((px - mx) * (px - mx) + (py - my) * (py - my));
                    }
                }
            }
        }
        dsum = block_reduce(dsum, 0, sh);
        if (cn > 0.0) ri = dsum / cn;
    }
    if (threadIdx.x == 0) {
        out[0] = ri;
        out[1] = DIM == 2 ? 0.5 * flat : sqrt(flat / 3.14159265358979323846);
        out[2] = cn;
    }
}

}  // namespace iblb
