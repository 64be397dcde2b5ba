// Learned preconditioner for the pressure solve (eq. (poisson)): a small 3-D
// convolutional network inside flexible CG.  The network, its training and the
// preconditioner application live here; the Krylov loop is in poisson.hip.
//
// Operator (linear and symmetric in the residual, so that a Krylov method sees a fixed
// symmetric positive definite preconditioner):
//   G = hsig(Wg * g)                     geometry gate, 16 channels, once per geometry
//   K x = W2 * ((W1 * x) . G)            conv 1 -> 16, gate, conv 16 -> 16
//   K^T y = W1^T * ((W2^T * y) . G)      the adjoint convolutions
//   z = D^-1 r + s K^T K (r / s),        s = RMS(r), D the diagonal of A = -L,
// "*" a zero-padded 3x3x3 cross-correlation, "^T *" its adjoint (flipped taps,
// transposed channels) and "." the per-channel product; g is the open-face fraction of
// the cell and hsig(v) = min(max(v/4 + 1/2, 0), 1), one clamped FMA.  Four 3x3x3 convolutions with 16 channels per application.
//
// MI355X design:
//  * activations channels-last in BF16: 16 channels = 32 bytes per cell, one 16-byte
//    load per lane feeds an MFMA operand;
//  * every convolution is an implicit GEMM on v_mfma_f32_16x16x32_bf16 with FP32
//    accumulation: M = 16 output channels, N = 16 cells along x, K = 32 = (two taps x
//    16 input channels), 14 k-steps per 3x3x3 stencil (2 for one input channel).  The
//    weights sit in registers for the whole block (A operand, 56 VGPRs); the input
//    tile with its halo (34 x 10 x 6 cells) is staged once in LDS as two 16-byte
//    half-cell planes so that the B-operand reads of 16 lanes are contiguous;
//  * the output D tile gives each lane 4 consecutive channels of one cell: one 8-byte
//    store per lane, 512 contiguous bytes per 16-cell tile; gating, the gate function and the
//    gradient of the gate are fused into that epilogue;
//  * an adjoint convolution is the same kernel with flipped, transposed packed weights;
//  * the weight gradient is an implicit GEMM over cells (K = cells of the tile): both
//    operands are staged channel-major in LDS, each block writes one partial 27x16x16
//    gradient and a second kernel sums the partials in block order (deterministic);
//  * blocks walk the tiles z-slowest through the XCD chunk map, so neighbouring tiles
//    (shared halos) run on one XCD and its L2.

#include <cmath>
#include <cstring>

#include "common.h"

namespace ibm {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int NWTS = IBM_CNN_NWEIGHTS;

// output tile of one convolution block and its halo
constexpr int CTX = 32, CTY = 8, CTZ = 4;
constexpr int HX = CTX + 2, HY = CTY + 2, HZ = CTZ + 2;
constexpr int HCELLS = HX * HY * HZ;      // 2040
constexpr int OCELLS = CTX * CTY * CTZ;   // 1024
constexpr int MTILES = OCELLS / 16;       // 16-cell MFMA column tiles per block
constexpr int WG_MAX_BLOCKS = 1024;       // weight-gradient partials

// epilogues of k_conv (acc = the FP32 convolution of the lane's 4 channels)
enum {
    EPI_BF16 = 0,     // out = bf16(acc)
    EPI_GATE = 1,     // out = bf16(acc . G); aux (optional) = bf16(acc)
    EPI_HSIG = 2,     // out = bf16(hsig(acc))
    EPI_BGATE = 3,    // out = bf16(acc . G); dG (float) = [dG +] acc . P
    EPI_F32 = 4,      // out = acc (float, COUT channels, stride ostride)
    EPI_COMBINE = 5   // marching 16 -> 1 only: the preconditioner's z (CombineIO)
};

// EPI_COMBINE: z = D^-1 r + s acc with D the diagonal of A = -L (open faces / dx^2),
// and the block's partial sums of <z, r> and <z, rp> (rp may be null) in cpart[b] and
// cpart[nblocks + b]
struct CombineIO {
    const float* r;
    const float* rp;
    const uint8_t* pcode;
    const double* s_in;
    double dx2;
    float* z;
    double* cpart;
    float wr;   // non-zero: z = D^-1 (r + wr rp) + s net (the smoothed form's z2), dots unused
};

// optional operands of the epilogues
struct ConvIO {
    const uint16_t* gate;   // G, cells x 16 BF16
    uint16_t* aux;          // EPI_GATE: pre-gate copy, or null
    const uint16_t* pre;    // EPI_BGATE: stored pre-gate activation P
    float* dg;              // EPI_BGATE: gate gradient accumulator, cells x 16
    int accum;              // EPI_BGATE: add to dg instead of overwriting
    int ostride;            // EPI_F32: floats per cell of out
};

__host__ __device__ constexpr int ksteps(int cin) { return cin == 16 ? 14 : (27 * cin + 31) / 32; }

// Tap order of the 16-channel k-steps.  Lane groups g = 0, 1 (h = 0) hold the first of
// the step's two taps, g = 2, 3 (h = 1) the second.  Taps are numbered
// 9 (dz + 1) + 3 (dy + 1) + (dx + 1).
//   s = 3 (dx + 1) + (dy + 1), s < 9:  (-1, dy, dx) and (+1, dy, dx)
//   s = 9 + (dy + 1):                  (0, dy, -1) and (0, dy, +1)
//   s = 12:                            (0, -1, 0) and (0, +1, 0)
//   s = 13:                            (0, 0, 0) and padding
// In the first twelve steps both taps of a pair have the same dy, so the B operand of
// input row i serves the output rows i - dy of all three dy (the marching kernel reads
// each such operand once for four output rows), and the second tap always lies a fixed
// distance from the first in the LDS halo planes.
__host__ __device__ constexpr int tap16(int s, int h) {
    return s < 9    ? (h ? 18 : 0) + 3 * (s % 3) + s / 3
           : s < 12 ? 9 + 3 * (s - 9) + (h ? 2 : 0)
           : s == 12 ? (h ? 16 : 10)
                     : (h ? -1 : 13);
}

// (tap, input channel) held by element e of lane group g in k-step s; tap = -1 for
// padding.  Used by the weight packing and by the B-operand gathers, so the two MFMA
// operands agree on k.  One input channel (a single k-step): group g < 3 holds taps
// q = 0..7 of plane dz = g - 1 (q = 3 (dy + 1) + (dx + 1)), group 3 holds q = 8 of
// the planes dz = -1, 0, +1 in its elements 0..2; again a lane's eight addresses are
// few base registers plus compile-time offsets.
template <int CIN>
__host__ __device__ inline void kmap(int s, int g, int e, int& tap, int& ci) {
    if (CIN == 16) {
        tap = tap16(s, g >> 1);
        ci = 8 * (g & 1) + e;
    } else if (CIN == 1) {
        tap = g < 3 ? 9 * g + e : (e < 3 ? 9 * e + 8 : -1);
        ci = 0;
    } else {
        const int k = 32 * s + 8 * g + e;
        tap = k / CIN;
        ci = k % CIN;
    }
    if (tap > 26) tap = -1;
}

// float -> bfloat16 bits, round to nearest, ties to even (the hardware conversion)
__device__ inline uint16_t f2bf(float f) {
    const __bf16 h = (__bf16)f;
    uint16_t u;
    __builtin_memcpy(&u, &h, 2);
    return u;
}
__device__ inline float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ inline int jcnt(uint8_t pc) { return __builtin_popcount((unsigned)(pc & 0x3F)) + 2 * (pc >> 6); }

// ------------------------------------------------------------------ weight packing

}  // namespace

struct PackDesc {
    int loff, lcin, lcout;   // layer: offset in the flat weights, its channels
    int bwd;                 // 0 forward conv, 1 backward-data conv (flipped, transposed)
    int cin, cout;           // channels of the conv as launched
    int ks, off;             // k-steps, offset in the packed array (elements)
    int ymode;               // 1: 16 -> 1 adjoint with A rows = dy + 1 (k_mconv, COUT = 1)
};

namespace {

// Packed A operand: for k-step s and lane l, 8 BF16 values W[row = l % 16][k(s, l / 16, e)].
__global__ void k_pack(const float* __restrict__ w, uint16_t* __restrict__ wp, PackDesc d) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= d.ks * 512) return;
    const int e = idx & 7, lane = (idx >> 3) & 63, s = idx >> 9;
    const int g = lane >> 4, row = lane & 15;
    int tap, ci;
    if (d.ymode) {
        // K = (dz, dx) pairs x 16 channels in 5 steps, M = dy + 1 (rows 0..2):
        // s < 3: (-1, s - 1) | (+1, s - 1); s = 3: (0, -1) | (0, +1); s = 4: (0, 0) | padding
        const int h = g >> 1, dy = row - 1;
        int dz = 0, dx = 0;
        if (s < 3) {
            dz = h ? 1 : -1;
            dx = s - 1;
        } else if (s == 3) {
            dx = h ? 1 : -1;
        }
        tap = (row < 3 && !(s == 4 && h)) ? 9 * (dz + 1) + 3 * (dy + 1) + (dx + 1) : -1;
        ci = 8 * (g & 1) + e;
        float val = 0.0f;
        if (tap >= 0) val = w[d.loff + ((26 - tap) * d.lcin + 0) * d.lcout + ci];
        wp[d.off + idx] = f2bf(val);
        return;
    }
    if (d.cin == 16)
        kmap<16>(s, g, e, tap, ci);
    else if (d.cin == 2)
        kmap<2>(s, g, e, tap, ci);
    else
        kmap<1>(s, g, e, tap, ci);
    float val = 0.0f;
    if (tap >= 0 && row < d.cout && ci < d.cin) {
        const float* wl = w + d.loff;
        if (!d.bwd)
            val = wl[(tap * d.lcin + ci) * d.lcout + row];
        else   // backward conv: input channel = layer output channel, output = layer input
            val = wl[((26 - tap) * d.lcin + row) * d.lcout + ci];
    }
    wp[d.off + idx] = f2bf(val);
}

// ------------------------------------------------------------------ convolution

__device__ inline void tile_of(int b, int nb, int ntx, int nty, int& tx, int& ty, int& tz) {
    const int t = xcd_chunk(b, nb);
    tx = t % ntx;
    ty = (t / ntx) % nty;
    tz = t / (ntx * nty);
}

__device__ inline void unpack4(uint2 w, float (&f)[4]) {
    f[0] = bf2f((uint16_t)(w.x & 0xFFFFu));
    f[1] = bf2f((uint16_t)(w.x >> 16));
    f[2] = bf2f((uint16_t)(w.y & 0xFFFFu));
    f[3] = bf2f((uint16_t)(w.y >> 16));
}
// two floats -> a BF16 pair (round to nearest even; a in the low half): one
// v_cvt_pk_bf16_f32
__device__ inline uint32_t pack2(float a, float b) {
    typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
    typedef float f32x2 __attribute__((ext_vector_type(2)));
    const bf16x2 h = __builtin_convertvector(f32x2{a, b}, bf16x2);
    uint32_t u;
    __builtin_memcpy(&u, &h, 4);
    return u;
}
__device__ inline uint2 pack4(const float (&f)[4]) { return make_uint2(pack2(f[0], f[1]), pack2(f[2], f[3])); }
// a, b rounded to BF16 (kept as floats)
__device__ inline void round2(float& a, float& b) {
    const uint32_t u = pack2(a, b);
    a = __uint_as_float(u << 16);
    b = __uint_as_float(u & 0xFFFF0000u);
}
// gate nonlinearity hsig(v) = v/4 + 1/2 clamped to [0, 1]: one FMA and a clamp (the
// logistic function it replaces cost two quarter-rate transcendentals per value and
// dominated the issue time of the gated convolutions)
__device__ inline float hsig(float x) { return fminf(fmaxf(fmaf(x, 0.25f, 0.5f), 0.0f), 1.0f); }

// One 3x3x3 convolution over an nx x ny x nz grid (zero padding): in = cells x CIN
// BF16 (channels-last), wp = packed weights, out per the epilogue (see EPI_*).
// sv (may be null): the solve's state; the kernel does nothing once it has converged.
template <int CIN, int COUT, int EPI>
__global__ void __launch_bounds__(256, 2) k_conv(int nx, int ny, int nz, const uint16_t* __restrict__ in,
                                                 const uint16_t* __restrict__ wp, void* __restrict__ out,
                                                 ConvIO io, const Solver* sv, int gate) {
    if (sv && stopped_before(sv, gate)) return;
    constexpr int KS = ksteps(CIN);
    constexpr int LDS_ELEMS = CIN == 16 ? 2 * HCELLS * 8 : HCELLS * CIN;
    __shared__ __attribute__((aligned(16))) uint16_t lds[LDS_ELEMS];
    const int ntx = (nx + CTX - 1) / CTX, nty = (ny + CTY - 1) / CTY;
    int tx, ty, tz;
    tile_of(blockIdx.x, gridDim.x, ntx, nty, tx, ty, tz);
    const int hx0 = tx * CTX - 1, hy0 = ty * CTY - 1, hz0 = tz * CTZ - 1;
    // stage the input tile with its halo (zero outside the grid)
    if (CIN == 16) {
        for (int q = threadIdx.x; q < 2 * HCELLS; q += 256) {
            const int cell = q >> 1, h = q & 1;
            const int hx = cell % HX, hy = (cell / HX) % HY, hz = cell / (HX * HY);
            const int gx = hx0 + hx, gy = hy0 + hy, gz = hz0 + hz;
            uint4 v = make_uint4(0u, 0u, 0u, 0u);
            if (gx >= 0 && gx < nx && gy >= 0 && gy < ny && gz >= 0 && gz < nz) {
                const long long c = (long long)gx + (long long)nx * ((long long)gy + (long long)ny * gz);
                v = *reinterpret_cast<const uint4*>(in + c * 16 + h * 8);
            }
            *reinterpret_cast<uint4*>(&lds[(h * HCELLS + cell) * 8]) = v;
        }
    } else {
        for (int cell = threadIdx.x; cell < HCELLS; cell += 256) {
            const int hx = cell % HX, hy = (cell / HX) % HY, hz = cell / (HX * HY);
            const int gx = hx0 + hx, gy = hy0 + hy, gz = hz0 + hz;
            const bool ok = gx >= 0 && gx < nx && gy >= 0 && gy < ny && gz >= 0 && gz < nz;
            const long long c = ok ? (long long)gx + (long long)nx * ((long long)gy + (long long)ny * gz) : 0;
#pragma unroll
            for (int ci = 0; ci < CIN; ++ci) lds[cell * CIN + ci] = ok ? in[c * CIN + ci] : (uint16_t)0;
        }
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int j = lane & 15, g = lane >> 4;
    bf16x8 wa[KS];
#pragma unroll
    for (int s = 0; s < KS; ++s) wa[s] = *reinterpret_cast<const bf16x8*>(wp + ((long long)s * 64 + lane) * 8);
    __syncthreads();
    for (int m = wv; m < MTILES; m += 4) {
        const int xg = m & 1, oy = (m >> 1) & (CTY - 1), oz = m >> 4;
        const int ox = xg * 16 + j;
        f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int s = 0; s < KS; ++s) {
            bf16x8 bv;
            if (CIN == 16) {
                int tap = tap16(s, g >> 1);
                if (tap < 0) tap = 13;   // padding slot: its weights are zero
                const int dz = tap / 9 - 1, dy = (tap / 3) % 3 - 1, dx = tap % 3 - 1;
                const int hc = (ox + 1 + dx) + HX * ((oy + 1 + dy) + HY * (oz + 1 + dz));
                bv = *reinterpret_cast<const bf16x8*>(&lds[((g & 1) * HCELLS + hc) * 8]);
            } else {
                uint16_t tmp[8];
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    int tap, ci;
                    kmap<CIN>(s, g, e, tap, ci);
                    uint16_t v = 0;
                    if (tap >= 0) {
                        const int dz = tap / 9 - 1, dy = (tap / 3) % 3 - 1, dx = tap % 3 - 1;
                        const int hc = (ox + 1 + dx) + HX * ((oy + 1 + dy) + HY * (oz + 1 + dz));
                        v = lds[hc * CIN + ci];
                    }
                    tmp[e] = v;
                }
                __builtin_memcpy(&bv, tmp, 16);
            }
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wa[s], bv, acc, 0, 0, 0);
        }
        // lane holds output channels 4g .. 4g+3 of cell (ox, oy, oz)
        const int gx = tx * CTX + ox, gy = ty * CTY + oy, gz = tz * CTZ + oz;
        if (gx < nx && gy < ny && gz < nz) {
            const long long c = (long long)gx + (long long)nx * ((long long)gy + (long long)ny * gz);
            if (EPI == EPI_F32) {
                if (g == 0) {
                    float* of = static_cast<float*>(out);
#pragma unroll
                    for (int r = 0; r < COUT; ++r) of[c * io.ostride + r] = acc[r];
                }
            } else {
                float v[4] = {acc[0], acc[1], acc[2], acc[3]};
                const long long o16 = c * 16 + 4 * g;
                if (EPI == EPI_HSIG) {
#pragma unroll
                    for (int r = 0; r < 4; ++r) v[r] = hsig(v[r]);
                } else if (EPI == EPI_GATE || EPI == EPI_BGATE) {
                    float gt[4];
                    unpack4(*reinterpret_cast<const uint2*>(io.gate + o16), gt);
                    if (EPI == EPI_GATE && io.aux) *reinterpret_cast<uint2*>(io.aux + o16) = pack4(v);
                    if (EPI == EPI_BGATE) {
                        float pr[4];
                        unpack4(*reinterpret_cast<const uint2*>(io.pre + o16), pr);
                        float4 d = io.accum ? *reinterpret_cast<const float4*>(io.dg + o16) : make_float4(0.f, 0.f, 0.f, 0.f);
                        d.x += v[0] * pr[0];
                        d.y += v[1] * pr[1];
                        d.z += v[2] * pr[2];
                        d.w += v[3] * pr[3];
                        *reinterpret_cast<float4*>(io.dg + o16) = d;
                    }
#pragma unroll
                    for (int r = 0; r < 4; ++r) v[r] *= gt[r];
                }
                *reinterpret_cast<uint2*>(static_cast<uint16_t*>(out) + o16) = pack4(v);
            }
        }
    }
}

// Marching form of a convolution for the solver's preconditioner applications.
// A block owns a 32 x 8 output tile in x-y and walks a slab of mz planes in z.  The
// input planes z-1, z, z+1 (34 x 10 cells with halo) sit in a ring of four LDS planes
// (two 16-byte half-cell planes each, HPC cells apart); plane z+2, loaded into
// registers while plane z is computed (one iteration earlier in the 16 -> 1 kernels,
// which then have plane z+3 in flight), is written to the free ring slot afterwards
// (one barrier per plane).  Each wave owns one
// 16-cell half of four output rows: four MFMA tiles, four independent accumulator
// chains, and each B operand read from LDS feeds up to three of them (tap16).
// EPI_BF16 as in k_conv; EPI_GATE computes the gate hsig(Wg * g) of its output cells on
// the fly (one more MFMA per tile from a ring of geometry planes) instead of reading a
// stored gate; EPI_F32 and EPI_COMBINE are the 16 -> 1 forms.
constexpr int PX = CTX + 2, PY = CTY + 2;    // 34 x 10 halo plane
constexpr int PCELLS = PX * PY;              // 340
constexpr int PCHUNK = (2 * PCELLS + 255) / 256;   // 16-byte chunks per thread per plane (CIN = 16)
constexpr int PSCAL = (PCELLS + 255) / 256;        // cells per thread per plane (1-channel planes)
// Stride of the two half-cell planes of a 16-channel ring slot, in cells: padded so
// that it is a multiple of 256 bytes.  The B-operand read of lane groups 0 and 1 (the
// two halves of the same cells) then falls on the same LDS banks at the same offset,
// which is conflict-free; at the unpadded 5440 bytes (64 mod 256) every 16-byte read
// takes extra bank-conflict cycles (measured with SQ_LDS_BANK_CONFLICT).
constexpr int HPC = 352;
static_assert(HPC >= PCELLS && (HPC * 16) % 256 == 0, "half-plane stride");

// halo-plane cell of in-plane tap q = 3 (dy + 1) + (dx + 1), relative to the cell at
// (dx, dy) = (-1, -1) of the output cell
__host__ __device__ constexpr int qcell(int q) { return q % 3 + PX * (q / 3); }

// in-plane cell of tap q = 3 (dy + 1) + (dx + 1) of a plane W cells wide, relative to
// the (dx, dy) = (-1, -1) neighbour
template <int W>
__host__ __device__ constexpr int qcellw(int q) { return q % 3 + W * (q / 3); }

// Per-lane cell offsets of the kmap<1> gathers from a ring of four 1-channel planes of
// `cells` cells, W wide, around plane p: element e of the lane reads cell
// a[e] + qcellw<W>(e) + (offset of its output cell).  cb = the output cell's (-1, -1)
// neighbour in the plane.
template <int W>
__device__ __forceinline__ void kmap1_cells(int p, int g, int cb, int cells, int (&a)[8]) {
    const int base = cb + ((p + (g < 3 ? g : 2) + 3) & 3) * cells;
#pragma unroll
    for (int e = 0; e < 8; ++e) a[e] = base;
#pragma unroll
    for (int e = 0; e < 3; ++e)
        if (g == 3) a[e] = cb + ((p + e + 3) & 3) * cells + qcellw<W>(8) - qcellw<W>(e);
}

// 16 -> 16 convolution of one plane from a ring of four 16-channel halo planes (34 x 10
// cells, two half-cell planes HPC cells apart, ring slots (z & 3) of the planes z - 1,
// z, z + 1 in sl0, sl1, sl2) into the wave's four accumulators: output rows r0 .. r0 + 3
// of one 16-cell x half, cb = halo cell of the lane's column at dx = -1 in halo row r0.
// The B operands come in five groups: the dz-pair steps of dx = -1, 0, +1 (halo rows
// r0 .. r0 + 5 each), the dx-pair steps (same rows), and the dy-pair and centre steps
// (four each).  The B operand of halo row r0 + ii feeds output row r0 + rr through the
// step of dy = ii - rr - 1; every chain accumulates its steps in increasing s, as k_conv
// does.  Group k + 1 is loaded while group k is multiplied.
__device__ __forceinline__ void conv16_plane(const uint16_t* ring, int cb, int g, int sl0, int sl1, int sl2,
                                             const bf16x8 (&wa)[14], f32x4 (&acc)[4]) {
    constexpr int PLANE = 2 * HPC * 8;
    const int h = g >> 1, hb = (g & 1) * HPC;
    const uint16_t* b0 = ring + (hb + cb) * 8 + (h ? sl2 : sl0) * PLANE;   // dz = -1 | +1
    const uint16_t* bx = ring + (hb + cb + 2 * h) * 8 + sl1 * PLANE;       // dx = -1 | +1
    const uint16_t* by = ring + (hb + cb + 2 * PX * h) * 8 + sl1 * PLANE;  // dy = -1 | +1
    const uint16_t* bc = ring + (hb + cb) * 8 + sl1 * PLANE;               // centre
    // six halo rows from base P (stride PX cells) starting at cell offset c0
    auto load6 = [&](const uint16_t* P, int c0, bf16x8 (&B)[6]) {
#pragma unroll
        for (int k = 0; k < 6; ++k) B[k] = *reinterpret_cast<const bf16x8*>(P + (k * PX + c0) * 8);
    };
    // steps s0 + dy + 1: dy outer so that consecutive MFMAs go to four different
    // accumulators (each still takes its steps in increasing s)
    auto mma6 = [&](int s0, const bf16x8 (&B)[6]) {
#pragma unroll
        for (int dyi = 0; dyi < 3; ++dyi) {
#pragma unroll
            for (int rr = 0; rr < 4; ++rr)
                acc[rr] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wa[s0 + dyi], B[rr + dyi], acc[rr], 0, 0, 0);
        }
    };
    bf16x8 Ba[6], Bb[6], Bd[4], Be[4];
    load6(b0, 0, Ba);
    load6(b0, 1, Bb);
    mma6(0, Ba);
    load6(b0, 2, Ba);
    mma6(3, Bb);
    load6(bx, 0, Bb);
    mma6(6, Ba);
#pragma unroll
    for (int rr = 0; rr < 4; ++rr) {
        Bd[rr] = *reinterpret_cast<const bf16x8*>(by + (rr * PX + 1) * 8);
        Be[rr] = *reinterpret_cast<const bf16x8*>(bc + ((rr + 1) * PX + 1) * 8);
    }
    mma6(9, Bb);
#pragma unroll
    for (int rr = 0; rr < 4; ++rr)
        acc[rr] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wa[12], Bd[rr], acc[rr], 0, 0, 0);
#pragma unroll
    for (int rr = 0; rr < 4; ++rr)
        acc[rr] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wa[13], Be[rr], acc[rr], 0, 0, 0);
}

// 16 -> 1 convolution of one plane (PV_W1TY packing): the A rows are m = dy + 1, K runs
// over (dz, dx) pairs x 16 channels in five steps (s < 3: dz = -1 | +1 at dx = s - 1;
// s = 3: dx = -1 | +1 in plane z; s = 4: the centre column and padding), so one MFMA
// chain per halo row ii = 0 .. 5 of the wave gives d[ii][m] = the part of every output
// row r0 + ii - m.  Lane group 0 then holds, per output row rr, the three parts of its
// cell: o[rr] = d[rr][0] + d[rr + 1][1] + d[rr + 2][2].  30 MFMAs for four rows instead
// of 56 with a single useful A row.
__device__ __forceinline__ void conv16to1_plane(const uint16_t* ring, int cb, int g, int sl0, int sl1, int sl2,
                                                const bf16x8 (&wa)[5], float (&o)[4]) {
    constexpr int PLANE = 2 * HPC * 8;
    const int h = g >> 1, hb = (g & 1) * HPC;
    const uint16_t* b0 = ring + (hb + cb) * 8 + (h ? sl2 : sl0) * PLANE;   // dz = -1 | +1
    const uint16_t* bx = ring + (hb + cb + 2 * h) * 8 + sl1 * PLANE;       // dx = -1 | +1
    const uint16_t* bc = ring + (hb + cb) * 8 + sl1 * PLANE;               // centre
    f32x4 d[6];
    __builtin_amdgcn_iglp_opt(0);   // interleave the B reads with the MFMAs (measured: helps here only)
#pragma unroll
    for (int ii = 0; ii < 6; ++ii) d[ii] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int s = 0; s < 5; ++s) {
        bf16x8 B[6];
#pragma unroll
        for (int ii = 0; ii < 6; ++ii) {
            const uint16_t* P = s < 3 ? b0 + (ii * PX + s) * 8 : (s == 3 ? bx + ii * PX * 8 : bc + (ii * PX + 1) * 8);
            B[ii] = *reinterpret_cast<const bf16x8*>(P);
        }
#pragma unroll
        for (int ii = 0; ii < 6; ++ii) d[ii] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wa[s], B[ii], d[ii], 0, 0, 0);
    }
#pragma unroll
    for (int rr = 0; rr < 4; ++rr) o[rr] = d[rr][0] + d[rr + 1][1] + d[rr + 2][2];
}

// Prefetch registers of one plane of the march: the thread's chunks of an input plane
// (and geometry plane for EPI_GATE), and for EPI_COMBINE the r, r_prev and face codes
// of the lane's output cells of one plane.  Two sets alternate, so that each load has
// two plane iterations to arrive (the light kernels of the march otherwise wait on HBM
// latency every plane).
struct MPre {
    uint4 pre[PCHUNK];
    uint16_t preg[PSCAL];
    float er, erp;   // EPI_COMBINE: r and r_prev of the lane's output cell (row g)
    uint8_t epc;     // and its face code
};

// The march of a 16-channel input (see above): COUT = 16 (EPI_BF16, EPI_GATE) or
// COUT = 1 (EPI_F32, EPI_COMBINE; conv16to1_plane with the PV_W1TY packing).
template <int COUT, int EPI>
__global__ void __launch_bounds__(256, 3) k_mconv(int nx, int ny, int nz, int mz, const uint16_t* __restrict__ in,
                                                  const uint16_t* __restrict__ wp, void* __restrict__ out,
                                                  const uint16_t* __restrict__ gsrc, const uint16_t* __restrict__ wgp,
                                                  const Solver* sv, int gate, CombineIO cio) {
    static_assert(COUT == 16 || COUT == 1, "marching convolution: 16 or 1 output channels");
    static_assert((EPI == EPI_COMBINE || EPI == EPI_F32) == (COUT == 1), "epilogue / output channels");
    if (sv && stopped_before(sv, gate)) return;
    constexpr int KS = COUT == 1 ? 5 : 14;
    constexpr int PLANE = 2 * HPC * 8;   // uint16 per ring plane
    __shared__ __attribute__((aligned(16))) uint16_t ring[4 * PLANE];
    // EPI_GATE: geometry planes as row pairs, cell c holding g(c) (low half) and g of the
    // cell one row below (high half), so that one 4-byte gather serves two output rows
    __shared__ uint32_t gring[EPI == EPI_GATE ? 4 * PCELLS : 1];
    const int ntx = (nx + CTX - 1) / CTX, nty = (ny + CTY - 1) / CTY;
    const int nslab = (nz + mz - 1) / mz;
    const int t = xcd_chunk(blockIdx.x, gridDim.x);
    const int tx = t % ntx, ty = (t / ntx) % nty, tzs = t / (ntx * nty);
    if (tzs >= nslab) {
        if (EPI == EPI_COMBINE && threadIdx.x == 0) cio.cpart[blockIdx.x] = cio.cpart[gridDim.x + blockIdx.x] = 0.0;
        return;
    }
    const int x0 = tx * CTX - 1, y0 = ty * CTY - 1;
    const int z0 = tzs * mz, z1 = min(nz, z0 + mz);
    const long long plane = (long long)nx * ny;
    __shared__ float invf[EPI == EPI_COMBINE ? 16 : 1];   // dx^2 / (open faces + 2 outlets)
    __shared__ double shr[EPI == EPI_COMBINE ? 8 : 1];
    if (EPI == EPI_COMBINE && threadIdx.x < 16)
        invf[threadIdx.x] = threadIdx.x ? (float)(cio.dx2 / (double)threadIdx.x) : 0.0f;
    const float sc = EPI == EPI_COMBINE ? (float)*cio.s_in : 0.0f;
    double zsum[2] = {0.0, 0.0};
    // The thread's loads are the same in every plane: in-plane byte offsets of its
    // chunks (half cells of 8 channels) and, for the gate, of its geometry cells.  Plane
    // loads go through buffer resources sized to the plane, so that a load at an offset
    // past its end returns zero: halo cells outside the grid (and threads without a
    // chunk) take offset OOB, and planes outside the grid get an empty resource.  The
    // host keeps nx * ny * 32 below 2^31.
    constexpr int OOB = 0x7FFFFFF0;
    constexpr int RSRC3 = 0x00020000;   // word 3 of a raw buffer resource on this target
    int o16[PCHUNK], o1[PSCAL];
#pragma unroll
    for (int k = 0; k < PCHUNK; ++k) {
        const int q = threadIdx.x + 256 * k;
        const int cell = q >> 1;
        int o = OOB;
        if (cell < PCELLS) {
            const int gx = x0 + cell % PX, gy = y0 + cell / PX;
            if (gx >= 0 && gx < nx && gy >= 0 && gy < ny) o = ((gx + nx * gy) * 16 + (q & 1) * 8) * 2;
        }
        o16[k] = o;
    }
#pragma unroll
    for (int k = 0; k < PSCAL; ++k) {
        const int cell = threadIdx.x + 256 * k;
        int o = OOB;
        if (EPI == EPI_GATE && cell < PCELLS) {
            const int gx = x0 + cell % PX, gy = y0 + cell / PX;
            if (gx >= 0 && gx < nx && gy >= 0 && gy < ny) o = (gx + nx * gy) * 2;
        }
        o1[k] = o;
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int j = lane & 15, g = lane >> 4;
    // the wave's outputs: x half xh (16 cells) of the four rows r0 .. r0 + 3, one MFMA
    // tile (one accumulator chain) per row
    const int xh = wv & 1, r0 = 4 * (wv >> 1);
    const int gxo = tx * CTX + 16 * xh + j;   // the lane's output column
    // halo-plane cell of the lane's column at dx = -1 in halo row r0 (the row above the
    // wave's first output row)
    const int cb = j + 16 * xh + PX * r0;
    // loader: plane pz of the halo region into registers (zero outside the grid)
    auto load_plane = [&](int pz, MPre& R) {
        const bool zin = pz >= 0 && pz < nz;
        const long long pb = zin ? (long long)pz * plane : 0;
        const int bytes = zin ? (int)(plane * 2) : 0;   // of one channel
        if (EPI == EPI_GATE) {
            const __amdgpu_buffer_rsrc_t rg =
                __builtin_amdgcn_make_buffer_rsrc(const_cast<uint16_t*>(gsrc + pb), 0, bytes, RSRC3);
#pragma unroll
            for (int k = 0; k < PSCAL; ++k) R.preg[k] = __builtin_amdgcn_raw_buffer_load_b16(rg, o1[k], 0, 0);
        }
        const __amdgpu_buffer_rsrc_t ri =
            __builtin_amdgcn_make_buffer_rsrc(const_cast<uint16_t*>(in + pb * 16), 0, bytes * 16, RSRC3);
#pragma unroll
        for (int k = 0; k < PCHUNK; ++k) {
            const auto v = __builtin_amdgcn_raw_buffer_load_b128(ri, o16[k], 0, 0);
            R.pre[k] = make_uint4(v[0], v[1], v[2], v[3]);
        }
    };
    // EPI_COMBINE: r, r_prev and the face code of output row g of the wave's cells of
    // plane pz: every lane loads one cell, so the four rows take one load each per array
    // (the wave's combine epilogue is spread over its four lane groups)
    const int gye = ty * CTY + r0 + g;
    // the lane's output cell of row g within a plane (OOB outside the grid: buffer loads
    // there return zero, buffer stores are dropped)
    const int ecell = (gxo < nx && gye < ny) ? gxo + nx * gye : -1;
    auto load_epi = [&](int pz, MPre& R) {
        if (EPI != EPI_COMBINE) return;
        // branch-free: planes at or past z1 get empty resources (zeros)
        const bool zin = pz < z1;
        const long long pb = zin ? (long long)pz * plane : 0;
        const int cells = zin ? (int)plane : 0;
        const __amdgpu_buffer_rsrc_t rr_ =
            __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(cio.r + pb), 0, 4 * cells, RSRC3);
        const __amdgpu_buffer_rsrc_t rc_ =
            __builtin_amdgcn_make_buffer_rsrc(const_cast<uint8_t*>(cio.pcode + pb), 0, cells, RSRC3);
        const __amdgpu_buffer_rsrc_t rp_ = __builtin_amdgcn_make_buffer_rsrc(
            const_cast<float*>(cio.rp ? cio.rp + pb : cio.r), 0, cio.rp ? 4 * cells : 0, RSRC3);
        R.er = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rr_, ecell < 0 ? OOB : 4 * ecell, 0, 0));
        R.erp = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rp_, ecell < 0 ? OOB : 4 * ecell, 0, 0));
        R.epc = __builtin_amdgcn_raw_buffer_load_b8(rc_, ecell < 0 ? OOB : ecell, 0, 0);
    };
    // Output stores, branch-free and one plane late (as in k_mfwd): plane z's values wait
    // in `held` / `held1` and are stored right after the loads at the top of the next
    // plane's step, with loop-invariant offsets and a per-plane resource (an empty one
    // before the first plane).
    int so[4];
#pragma unroll
    for (int rr = 0; rr < 4; ++rr) {
        const int gy = ty * CTY + r0 + rr;
        so[rr] = (gxo < nx && gy < ny) ? ((gxo + nx * gy) * 16 + 4 * g) * 2 : OOB;
    }
    uint2 held[4];
#pragma unroll
    for (int rr = 0; rr < 4; ++rr) held[rr] = make_uint2(0u, 0u);
    float held1 = 0.0f;
    auto store_held = [&](int zp) {
        const bool any = zp >= z0;
        if constexpr (COUT == 16) {
            const __amdgpu_buffer_rsrc_t ro = __builtin_amdgcn_make_buffer_rsrc(
                static_cast<uint16_t*>(out) + (any ? (long long)zp * plane * 16 : 0), 0, any ? (int)(plane * 32) : 0,
                RSRC3);
#pragma unroll
            for (int rr = 0; rr < 4; ++rr) {
                typedef unsigned int v2u __attribute__((ext_vector_type(2)));
                const v2u w = {held[rr].x, held[rr].y};
                __builtin_amdgcn_raw_buffer_store_b64(w, ro, so[rr], 0, 0);
            }
        } else {
            float* dst = EPI == EPI_COMBINE ? cio.z : static_cast<float*>(out);
            const __amdgpu_buffer_rsrc_t ro = __builtin_amdgcn_make_buffer_rsrc(
                dst + (any ? (long long)zp * plane : 0), 0, any ? (int)(plane * 4) : 0, RSRC3);
            __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned int, held1), ro,
                                                  ecell < 0 ? OOB : 4 * ecell, 0, 0);
        }
    };
    auto store_plane = [&](int slot, const MPre& R) {
        if (EPI == EPI_GATE) {
            uint16_t* G16 = reinterpret_cast<uint16_t*>(gring + slot * PCELLS);
#pragma unroll
            for (int k = 0; k < PSCAL; ++k) {
                const int cell = threadIdx.x + 256 * k;
                if (cell < PCELLS) {
                    G16[2 * cell] = R.preg[k];
                    if (cell >= PX) G16[2 * (cell - PX) + 1] = R.preg[k];
                    else G16[2 * (cell + (PY - 1) * PX) + 1] = 0;   // last row: no row below
                }
            }
        }
        uint16_t* P = ring + slot * PLANE;
#pragma unroll
        for (int k = 0; k < PCHUNK; ++k) {
            const int q = threadIdx.x + 256 * k;
            if (q < 2 * PCELLS) *reinterpret_cast<uint4*>(&P[((q & 1) * HPC + (q >> 1)) * 8]) = R.pre[k];
        }
    };
    bf16x8 wa[KS];
#pragma unroll
    for (int s = 0; s < KS; ++s) wa[s] = *reinterpret_cast<const bf16x8*>(wp + ((long long)s * 64 + lane) * 8);
    bf16x8 wg;
    if (EPI == EPI_GATE) wg = *reinterpret_cast<const bf16x8*>(wgp + (long long)lane * 8);
    // The 16 -> 1 kernels (30 MFMAs per plane) keep two planes in flight; the 16 -> 16
    // kernels (56 to 60 MFMAs per plane, register-bound) one.
    constexpr bool DEEP = COUT == 1;
    // one plane z of the march: DEEP: planes z + 3 (input) and z + 1 (combine operands)
    // load into L while plane z is computed, S holds plane z + 2 and plane z's combine
    // operands; otherwise L = S and plane z + 2 loads into it.  Plane z + 2 is stored
    // into the ring slot of plane z - 2 after the compute.
    auto step = [&](int z, MPre& L, const MPre& S) {
        load_plane(z + (DEEP ? 3 : 2), L);
        load_epi(z + 1, L);
        store_held(z - 1);
        // ring slots of the planes z - 1, z, z + 1
        const int sl0 = (z + 3) & 3, sl1 = z & 3, sl2 = (z + 1) & 3;
        // gate of the output cells, BF16(hsig(Wg * g)) as the stored gate: gathered
        // first so that its LDS latency hides behind the convolution; computed for every
        // row (out-of-grid cells read zeros) so that no MFMA sits in a branch.  kmap<1>
        // gathers: element e of the lane reads cell a1[e] + qcell(e) + PX rr of the ring.
        f32x4 gacc[4];
        if (EPI == EPI_GATE) {
            int a1[8];
            kmap1_cells<PX>(z, g, cb, PCELLS, a1);
#pragma unroll
            for (int pp = 0; pp < 2; ++pp) {   // output rows 2 pp and 2 pp + 1
                uint32_t w8[8], lo[4], hi[4];
#pragma unroll
                for (int e = 0; e < 8; ++e) w8[e] = gring[a1[e] + qcell(e) + PX * 2 * pp];
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    lo[e] = __builtin_amdgcn_perm(w8[2 * e + 1], w8[2 * e], 0x05040100u);
                    hi[e] = __builtin_amdgcn_perm(w8[2 * e + 1], w8[2 * e], 0x07060302u);
                }
                bf16x8 b0, b1;
                __builtin_memcpy(&b0, lo, 16);
                __builtin_memcpy(&b1, hi, 16);
                gacc[2 * pp] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wg, b0, f32x4{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
                gacc[2 * pp + 1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wg, b1, f32x4{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
            }
        }
        f32x4 acc[4];
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) acc[rr] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
        float o1[4] = {0.0f, 0.0f, 0.0f, 0.0f};   // COUT = 1: the output of lane group 0
        if constexpr (COUT == 1)
            conv16to1_plane(ring, cb, g, sl0, sl1, sl2, wa, o1);
        else
            conv16_plane(ring, cb, g, sl0, sl1, sl2, wa, acc);
        float gate4[4][4];
        if (EPI == EPI_GATE) {
#pragma unroll
            for (int rr = 0; rr < 4; ++rr) {
#pragma unroll
                for (int r = 0; r < 4; ++r) gate4[rr][r] = hsig(gacc[rr][r]);
                round2(gate4[rr][0], gate4[rr][1]);
                round2(gate4[rr][2], gate4[rr][3]);
            }
        }
        if (EPI == EPI_COMBINE || EPI == EPI_F32) {
            // output row g of the lane's column: lane group 0 holds the four rows' sums
            const float t1 = __shfl(o1[1], j), t2 = __shfl(o1[2], j), t3 = __shfl(o1[3], j);
            const float om = g == 0 ? o1[0] : (g == 1 ? t1 : (g == 2 ? t2 : t3));
            if (EPI == EPI_COMBINE) {
                // outside the grid r = r_prev = 0 and the code is 0: no contribution
                const float rin = cio.wr != 0.0f ? fmaf(cio.wr, S.erp, S.er) : S.er;
                const float zi = invf[jcnt(S.epc)] * rin + sc * om;
                held1 = zi;
                zsum[0] += (double)zi * (double)S.er;
                zsum[1] += (double)zi * (double)S.erp;
            } else {
                held1 = om;
            }
        }
        if constexpr (COUT == 16) {
#pragma unroll
            for (int rr = 0; rr < 4; ++rr) {
                float v[4] = {acc[rr][0], acc[rr][1], acc[rr][2], acc[rr][3]};
                if (EPI == EPI_GATE) {
#pragma unroll
                    for (int r = 0; r < 4; ++r) v[r] *= gate4[rr][r];
                }
                held[rr] = pack4(v);
            }
        }
        store_plane((z + 2) & 3, S);   // slot of plane z - 2, last read for plane z - 1
        __syncthreads();
    };
    // prologue: planes z0 - 1, z0, z0 + 1 into ring slots (z & 3); DEEP: plane z0 + 2 and
    // the combine operands of plane z0 into registers
    MPre A, B;
    for (int pz = z0 - 1; pz <= z0 + 1; ++pz) {
        load_plane(pz, A);
        store_plane(pz & 3, A);
    }
    if (DEEP) {
        load_plane(z0 + 2, A);
        load_epi(z0, A);
    }
    __syncthreads();
    if constexpr (DEEP) {
        for (int z = z0; z < z1; z += 2) {
            step(z, B, A);
            if (z + 1 < z1) step(z + 1, A, B);
        }
    } else {
        for (int z = z0; z < z1; ++z) step(z, A, A);
    }
    store_held(z1 - 1);
    if (EPI == EPI_COMBINE) {
        block_reduce<2>(zsum, shr);
        if (threadIdx.x == 0) {
            cio.cpart[blockIdx.x] = zsum[0];
            cio.cpart[gridDim.x + blockIdx.x] = zsum[1];
        }
    }
}

// The combine epilogue's block partials (nb of them per sum, in cpart) summed in block
// order into the solver's reduction slots: the total in entry 0, zeros in entries
// 1 .. nparts - 1 (the consumers sum nparts entries of a slot).  zrp_slot < 0: none.
__global__ void __launch_bounds__(NT) k_relay(const double* __restrict__ cpart, int nb, double* __restrict__ partials,
                                              int nparts, int zr_slot, int zrp_slot, const Solver* sv, int gate) {
    if (sv && stopped_before(sv, gate)) return;
    __shared__ double sh[8];
    double v[2] = {0.0, 0.0};
    for (int b = threadIdx.x; b < nb; b += NT) {
        v[0] += cpart[b];
        v[1] += cpart[nb + b];
    }
    block_reduce<2>(v, sh);
    for (int b = threadIdx.x; b < nparts; b += NT) {
        partials[zr_slot * MAX_BLOCKS + b] = b ? 0.0 : v[0];
        if (zrp_slot >= 0) partials[zrp_slot * MAX_BLOCKS + b] = b ? 0.0 : v[1];
    }
}

// Forward half y = K x = W2 * ((W1 * x) . G) of the preconditioner in one marching
// pass.  The gated first convolution a1 = (W1 * x) . hsig(Wg * g) is recomputed
// plane by plane on the 34 x 10 halo region the second convolution needs, from an LDS
// ring of (x, g) pairs over 36 x 12 cells, and kept in a 16-channel LDS ring
// (the layout of k_mconv's); only y goes to HBM.  Both convolutions take the roundings
// and k-step orders of k_mconv<1, 16, EPI_GATE> followed by k_mconv<16, 16, EPI_BF16>,
// so y is the same bit for bit.  a1 is zero outside the grid (the second convolution's
// zero padding).  Pipeline at plane z: x, g of plane z + 4 load into registers, a1 of
// plane z + 2 is made from x, g of the planes z + 1 .. z + 3, y of plane z is made from
// a1 of the planes z - 1 .. z + 1, and x, g of plane z + 4 go to the ring slot of plane
// z; one barrier per plane.
constexpr int QX = CTX + 4, QY = CTY + 4;    // 36 x 12
constexpr int QCELLS = QX * QY;              // 432
constexpr int QSCAL = (QCELLS + 255) / 256;  // cells per thread per plane
constexpr int NA1 = (PCELLS + 15) / 16;      // 16-cell MFMA tiles of the 34 x 10 region (22)
constexpr int NA1W = (NA1 + 3) / 4;          // of them per wave, at most

// RIN: the input is the solver's FP32 residual r and the kernel forms x = BF16(r / s)
// itself (as r times 1/s in FP64), s^2 = (sum of the nparts partials of <r,r> in
// rpart) / cells, as k_input does
// (block 0 stores s in s_out for the combining step); otherwise xin is x (BF16).
template <bool RIN>
__global__ void __launch_bounds__(256, 3) k_mfwd(int nx, int ny, int nz, int mz, const void* __restrict__ xin,
                                                 const uint16_t* __restrict__ gsrc,
                                                 const uint16_t* __restrict__ w1p, const uint16_t* __restrict__ wgp,
                                                 const uint16_t* __restrict__ w2p, uint16_t* __restrict__ out,
                                                 const double* __restrict__ rpart, int nparts, double* __restrict__ s_out,
                                                 const Solver* sv, int gate) {
    if (sv && stopped_before(sv, gate)) return;
    constexpr int PLANE = 2 * HPC * 8;   // uint16 per 16-channel ring plane
    constexpr int OOB = 0x7FFFFFF0;
    constexpr int RSRC3 = 0x00020000;
    __shared__ __attribute__((aligned(16))) uint16_t ring[4 * PLANE];
    __shared__ uint32_t xgring[4 * QCELLS];   // per cell: x (low half), g (high half)
    const int ntx = (nx + CTX - 1) / CTX, nty = (ny + CTY - 1) / CTY;
    const int nslab = (nz + mz - 1) / mz;
    const int t = xcd_chunk(blockIdx.x, gridDim.x);
    const int tx = t % ntx, ty = (t / ntx) % nty, tzs = t / (ntx * nty);
    if (tzs >= nslab) return;
    const int z0 = tzs * mz, z1 = min(nz, z0 + mz);
    const long long plane = (long long)nx * ny;
    double rinv = 0.0;   // RIN: 1 / s (0 when r = 0)
    if (RIN) {
        __shared__ double sh[4];
        double v[1] = {0.0};
        for (int b = threadIdx.x; b < nparts; b += NT) v[0] += rpart[b];
        block_reduce<1>(v, sh);
        const double rs = sqrt(v[0] / (double)(plane * nz));
        rinv = rs > 0.0 ? 1.0 / rs : 0.0;
        if (blockIdx.x == 0 && threadIdx.x == 0) *s_out = rs;
    }
    // loader of the 36 x 12 region of x and g (byte offsets within a plane of g; OOB
    // outside the grid, where the buffer load returns zero)
    const int qx0 = tx * CTX - 2, qy0 = ty * CTY - 2;
    int oq[QSCAL];
#pragma unroll
    for (int k = 0; k < QSCAL; ++k) {
        const int cell = threadIdx.x + 256 * k;
        int o = OOB;
        if (cell < QCELLS) {
            const int gx = qx0 + cell % QX, gy = qy0 + cell / QX;
            if (gx >= 0 && gx < nx && gy >= 0 && gy < ny) o = (gx + nx * gy) * 2;
        }
        oq[k] = o;
    }
    uint16_t px[QSCAL], pg[QSCAL];
    float pr[RIN ? QSCAL : 1];
    auto load_xg = [&](int pz) {
        const bool zin = pz >= 0 && pz < nz;
        const long long pb = zin ? (long long)pz * plane : 0;
        const int bytes = zin ? (int)(plane * 2) : 0;
        const __amdgpu_buffer_rsrc_t rg = __builtin_amdgcn_make_buffer_rsrc(const_cast<uint16_t*>(gsrc + pb), 0, bytes, RSRC3);
        if (RIN) {
            const __amdgpu_buffer_rsrc_t rx = __builtin_amdgcn_make_buffer_rsrc(
                const_cast<float*>(static_cast<const float*>(xin) + pb), 0, 2 * bytes, RSRC3);
#pragma unroll
            for (int k = 0; k < QSCAL; ++k)
                pr[k] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rx, oq[k] == OOB ? OOB : 2 * oq[k], 0, 0));
        } else {
            const __amdgpu_buffer_rsrc_t rx = __builtin_amdgcn_make_buffer_rsrc(
                const_cast<uint16_t*>(static_cast<const uint16_t*>(xin) + pb), 0, bytes, RSRC3);
#pragma unroll
            for (int k = 0; k < QSCAL; ++k) px[k] = __builtin_amdgcn_raw_buffer_load_b16(rx, oq[k], 0, 0);
        }
#pragma unroll
        for (int k = 0; k < QSCAL; ++k) pg[k] = __builtin_amdgcn_raw_buffer_load_b16(rg, oq[k], 0, 0);
    };
    auto store_xg = [&](int slot) {
#pragma unroll
        for (int k = 0; k < QSCAL; ++k) {
            const int cell = threadIdx.x + 256 * k;
            if (cell < QCELLS) {
                const uint16_t xv = RIN ? f2bf((float)((double)pr[k] * rinv)) : px[k];
                xgring[slot * QCELLS + cell] = (uint32_t)xv | ((uint32_t)pg[k] << 16);
            }
        }
    };
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int j = lane & 15, g = lane >> 4;
    const bf16x8 w1 = *reinterpret_cast<const bf16x8*>(w1p + (long long)lane * 8);
    const bf16x8 wg = *reinterpret_cast<const bf16x8*>(wgp + (long long)lane * 8);
    bf16x8 wa[14];
#pragma unroll
    for (int s = 0; s < 14; ++s) wa[s] = *reinterpret_cast<const bf16x8*>(w2p + ((long long)s * 64 + lane) * 8);
    // a1 tiles of the wave: tile wv + 4 i covers cells 16 (wv + 4 i) .. + 15 of the 34 x 10
    // region (row-major; cells 340 .. 351 are padding, gathered at a clamped cell and
    // written to the padding of the half planes).  Per tile: the lane's cell index in
    // the 36-wide x, g planes (at its (-1, -1) neighbour) and whether its cell is inside
    // the grid.
    // The gate's FMA constant carries the zero outside the grid: hsig(v) = clamp(v/4 + c)
    // with c = 1/2 inside and -1e30 outside, where the gate and so a1 become 0.
    int qb[NA1W];
    float gc[NA1W];
#pragma unroll
    for (int i = 0; i < NA1W; ++i) {
        const int c = 16 * (wv + 4 * i) + j;
        const int cc = c < PCELLS ? c : PCELLS - 1;
        const int cx = cc % PX, cy = cc / PX;
        qb[i] = cx + QX * cy;
        const int gx = tx * CTX - 1 + cx, gy = ty * CTY - 1 + cy;
        gc[i] = (c < PCELLS && gx >= 0 && gx < nx && gy >= 0 && gy < ny) ? 0.5f : -1e30f;
    }
    // a1 of plane p into its ring slot (zero outside the grid)
    auto make_a1 = [&](int p) {
        uint16_t* A = ring + (p & 3) * PLANE;
        if (p < 0 || p >= nz) {
            for (int q = threadIdx.x; q < 2 * HPC; q += 256)
                *reinterpret_cast<uint4*>(&A[q * 8]) = make_uint4(0u, 0u, 0u, 0u);
            return;
        }
        int a[8];
        kmap1_cells<QX>(p, g, 0, QCELLS, a);
#pragma unroll
        for (int i = 0; i < NA1W; ++i) {
            const int tt = wv + 4 * i;
            if (tt >= NA1) break;   // uniform in the wave
            // one 4-byte gather per tap; the two B operands are the low and high halves
            uint32_t xg8[8], bxw[4], bgw[4];
#pragma unroll
            for (int e = 0; e < 8; ++e) xg8[e] = xgring[a[e] + qb[i] + qcellw<QX>(e)];
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                bxw[e] = __builtin_amdgcn_perm(xg8[2 * e + 1], xg8[2 * e], 0x05040100u);
                bgw[e] = __builtin_amdgcn_perm(xg8[2 * e + 1], xg8[2 * e], 0x07060302u);
            }
            bf16x8 bx, bg;
            __builtin_memcpy(&bx, bxw, 16);
            __builtin_memcpy(&bg, bgw, 16);
            const f32x4 ax = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w1, bx, f32x4{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
            const f32x4 ag = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wg, bg, f32x4{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
            float gt[4], v[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) gt[r] = fminf(fmaxf(fmaf(ag[r], 0.25f, gc[i]), 0.0f), 1.0f);   // hsig
            round2(gt[0], gt[1]);
            round2(gt[2], gt[3]);
#pragma unroll
            for (int r = 0; r < 4; ++r) v[r] = ax[r] * gt[r];
            // lane (j, g): channels 4 g .. 4 g + 3 of cell 16 tt + j
            *reinterpret_cast<uint2*>(&A[((g >> 1) * HPC + 16 * tt + j) * 8 + 4 * (g & 1)]) = pack4(v);
        }
    };
    // prologue: x, g of the planes z0 - 2 .. z0 + 3 and a1 of z0 - 1 .. z0 + 1
    for (int pz = z0 - 2; pz <= z0; ++pz) {
        load_xg(pz);
        store_xg(pz & 3);
    }
    __syncthreads();
    for (int p = z0 - 1; p <= z0 + 1; ++p) {
        make_a1(p);
        load_xg(p + 2);
        store_xg((p + 2) & 3);
        __syncthreads();
    }
    const int xh = wv & 1, r0 = 4 * (wv >> 1);
    const int cb = j + 16 * xh + PX * r0;
    const int gx = tx * CTX + 16 * xh + j;
    // Output stores, branch-free and one plane late.  Each lane's four 8-byte stores use
    // loop-invariant byte offsets within a plane (OOB for cells outside the grid, where
    // the buffer store is dropped) and a per-plane resource.  Plane z's packed values
    // stay in `held` until the stores issued at the top of iteration z + 1 have read them
    // (they are overwritten only after that iteration's convolution), and those stores
    // are issued after the iteration's loads, so that waiting for the loads never waits
    // for a store and no register a store still reads is reused early.
    int so[4];
#pragma unroll
    for (int rr = 0; rr < 4; ++rr) {
        const int gy = ty * CTY + r0 + rr;
        so[rr] = (gx < nx && gy < ny) ? ((gx + nx * gy) * 16 + 4 * g) * 2 : OOB;
    }
    uint2 held[4];
#pragma unroll
    for (int rr = 0; rr < 4; ++rr) held[rr] = make_uint2(0u, 0u);
    // the stores of plane zp (an empty resource before the first plane: dropped)
    auto store_held = [&](int zp) {
        const bool any = zp >= z0;
        const __amdgpu_buffer_rsrc_t ro = __builtin_amdgcn_make_buffer_rsrc(
            out + (any ? (long long)zp * plane * 16 : 0), 0, any ? (int)(plane * 32) : 0, RSRC3);
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) {
            typedef unsigned int v2u __attribute__((ext_vector_type(2)));
            const v2u w = {held[rr].x, held[rr].y};
            __builtin_amdgcn_raw_buffer_store_b64(w, ro, so[rr], 0, 0);
        }
    };
    for (int z = z0; z < z1; ++z) {
        load_xg(z + 4);
        store_held(z - 1);
        make_a1(z + 2);
        f32x4 acc[4];
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) acc[rr] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
        conv16_plane(ring, cb, g, (z + 3) & 3, z & 3, (z + 1) & 3, wa, acc);
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) {
            float v[4] = {acc[rr][0], acc[rr][1], acc[rr][2], acc[rr][3]};
            held[rr] = pack4(v);
        }
        store_xg(z & 3);   // plane z + 4
        __syncthreads();
    }
    store_held(z1 - 1);
}

// Weight gradient of one layer: dW[t][ci][co] = sum over cells c of X[c + off_t][ci] dY[c][co].
// MFMA with M = co, N = ci, K = 32 cells of the tile.  Each block loops over tiles and
// writes its partial 27 x 16 x 16 sum (layout t*256 + ci*16 + co).
template <int CIN, int COUT>
__global__ void __launch_bounds__(256, 1) k_wgrad(int nx, int ny, int nz, const uint16_t* __restrict__ x,
                                                  const uint16_t* __restrict__ dy, float* __restrict__ part,
                                                  int ntiles) {
    __shared__ __attribute__((aligned(16))) uint16_t xs[CIN * HCELLS];
    __shared__ __attribute__((aligned(16))) uint16_t ds[COUT * OCELLS];
    const int ntx = (nx + CTX - 1) / CTX, nty = (ny + CTY - 1) / CTY;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int j = lane & 15, g = lane >> 4;
    f32x4 acc[7];
#pragma unroll
    for (int q = 0; q < 7; ++q) acc[q] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
        int tx, ty, tz;
        tile_of(t, ntiles, ntx, nty, tx, ty, tz);
        const int hx0 = tx * CTX - 1, hy0 = ty * CTY - 1, hz0 = tz * CTZ - 1;
        __syncthreads();   // previous tile's reads are done
        for (int cell = threadIdx.x; cell < HCELLS; cell += 256) {
            const int hx = cell % HX, hy = (cell / HX) % HY, hz = cell / (HX * HY);
            const int gx = hx0 + hx, gy = hy0 + hy, gz = hz0 + hz;
            const bool ok = gx >= 0 && gx < nx && gy >= 0 && gy < ny && gz >= 0 && gz < nz;
            const long long c = ok ? (long long)gx + (long long)nx * ((long long)gy + (long long)ny * gz) : 0;
#pragma unroll
            for (int ci = 0; ci < CIN; ++ci) xs[ci * HCELLS + cell] = ok ? x[c * CIN + ci] : (uint16_t)0;
        }
        for (int cell = threadIdx.x; cell < OCELLS; cell += 256) {
            const int ox = cell % CTX, oy = (cell / CTX) % CTY, oz = cell / (CTX * CTY);
            const int gx = hx0 + 1 + ox, gy = hy0 + 1 + oy, gz = hz0 + 1 + oz;
            const bool ok = gx < nx && gy < ny && gz < nz;
            const long long c = ok ? (long long)gx + (long long)nx * ((long long)gy + (long long)ny * gz) : 0;
#pragma unroll
            for (int co = 0; co < COUT; ++co) ds[co * OCELLS + cell] = ok ? dy[c * COUT + co] : (uint16_t)0;
        }
        __syncthreads();
        for (int kb = 0; kb < OCELLS; kb += 32) {
            // A operand: dY of channel j for the 8 cells kb + 8g .. kb + 8g + 7
            bf16x8 av;
            if (j < COUT) {
                av = *reinterpret_cast<const bf16x8*>(&ds[j * OCELLS + kb + 8 * g]);
            } else {
                const uint16_t z8[8] = {0, 0, 0, 0, 0, 0, 0, 0};
                __builtin_memcpy(&av, z8, 16);
            }
            const int k0 = kb + 8 * g;   // first of 8 cells, all in one tile row
            const int ox0 = k0 % CTX, oy = (k0 / CTX) % CTY, oz = k0 / (CTX * CTY);
#pragma unroll
            for (int q = 0; q < 7; ++q) {
                const int tap = wv + 4 * q;
                if (tap > 26) break;
                const int dz = tap / 9 - 1, dyy = (tap / 3) % 3 - 1, dx = tap % 3 - 1;
                uint16_t tmp[8];
                const int hc0 = (ox0 + 1 + dx) + HX * ((oy + 1 + dyy) + HY * (oz + 1 + dz));
#pragma unroll
                for (int e = 0; e < 8; ++e) tmp[e] = j < CIN ? xs[j * HCELLS + hc0 + e] : (uint16_t)0;
                bf16x8 bv;
                __builtin_memcpy(&bv, tmp, 16);
                acc[q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, acc[q], 0, 0, 0);
            }
        }
    }
    // lane holds D[co = 4g + r][ci = j] of each of its taps
    float* pb = part + (long long)blockIdx.x * (27 * 256);
#pragma unroll
    for (int q = 0; q < 7; ++q) {
        const int tap = wv + 4 * q;
        if (tap > 26) break;
#pragma unroll
        for (int r = 0; r < 4; ++r) pb[tap * 256 + j * 16 + 4 * g + r] = acc[q][r];
    }
}

// dW (layer layout [27][CIN][COUT]) = (accum ? dW : 0) + the block partials in block order
__global__ void k_wsum(const float* __restrict__ part, int nblocks, int cin, int cout, float* __restrict__ dw,
                       int accum) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= 27 * cin * cout) return;
    const int co = idx % cout, ci = (idx / cout) % cin, t = idx / (cout * cin);
    const int o = t * 256 + ci * 16 + co;
    float s = 0.0f;
    for (int b = 0; b < nblocks; ++b) s += part[(long long)b * (27 * 256) + o];
    dw[idx] = accum ? dw[idx] + s : s;
}

// ------------------------------------------------------------------ input, loss, Adam

// partial sums of f^2 (one per block)
template <class T>
__global__ void __launch_bounds__(NT) k_sumsq(long long n, const T* __restrict__ f, double* __restrict__ part) {
    __shared__ double sh[4];
    double v[1] = {0.0};
    for (long long i = (long long)blockIdx.x * NT + threadIdx.x; i < n; i += (long long)gridDim.x * NT) {
        const double a = (double)f[i];
        v[0] += a * a;
    }
    block_reduce<1>(v, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = v[0];
}

// Network input x = BF16(f / s) with s^2 = (sum of the partials of <f,f>) / n.  With a
// solver state the kernel does nothing once the solve has stopped before iteration it,
// and with `check` it stops the solve itself at iteration it when <f,f> <= tol2; s is
// stored for the combining step.
template <class T>
__global__ void __launch_bounds__(NT) k_input(long long n, const T* __restrict__ f, const double* __restrict__ part,
                                              int nparts, uint16_t* __restrict__ x, double* __restrict__ s_out,
                                              Solver* sv, int it, int check) {
    if (sv && stopped_before(sv, it)) return;
    __shared__ double sh[4];
    double v[1] = {0.0};
    for (int b = threadIdx.x; b < nparts; b += NT) v[0] += part[b];
    block_reduce<1>(v, sh);
    const double ff = v[0];
    if (sv && check) {
        if (!(ff == ff)) {
            if (blockIdx.x == 0 && threadIdx.x == 0) {
                sv->nan_seen = 1;
                sv->converged = 3;
                sv->iters = it;
                sv->stop_it = it;
            }
            return;
        }
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            sv->rr = ff;
            sv->iters = it;
        }
        if (ff <= sv->tol2) {
            if (blockIdx.x == 0 && threadIdx.x == 0) {
                sv->converged = 1;
                sv->stop_it = it;
            }
            return;
        }
    }
    const double s = sqrt(ff / (double)n);
    const double sinv = s > 0.0 ? 1.0 / s : 0.0;
    if (blockIdx.x == 0 && threadIdx.x == 0) *s_out = s;
    for (long long i = (long long)blockIdx.x * NT + threadIdx.x; i < n; i += (long long)gridDim.x * NT)
        x[i] = f2bf((float)((double)f[i] * sinv));
}

// geometry input: BF16(open pressure faces / 6)
__global__ void k_geom(long long n, const uint8_t* __restrict__ pcode, uint16_t* __restrict__ xg) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        xg[i] = f2bf((float)((double)__builtin_popcount((unsigned)(pcode[i] & 0x3F)) / 6.0));
}

// cells x 2 BF16 -> two single-channel planes
__global__ void k_split(long long n, const uint16_t* __restrict__ x2, uint16_t* __restrict__ a,
                        uint16_t* __restrict__ b) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
        a[i] = x2[2 * i];
        b[i] = x2[2 * i + 1];
    }
}

// gradient at the gate's pre-activation: BF16(dG . hsig'), hsig' = 1/4 where 0 < G < 1, else 0
__global__ void k_dpre(long long n16, const float* __restrict__ dg, const uint16_t* __restrict__ gt,
                       uint16_t* __restrict__ out) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += (long long)gridDim.x * blockDim.x) {
        const float gv = bf2f(gt[i]);
        out[i] = f2bf(dg[i] * ((gv > 0.0f && gv < 1.0f) ? 0.25f : 0.0f));
    }
}

// h = D^-1 f + s y (double)
__global__ void k_phat(long long n, double dx2, const double* __restrict__ f, const uint8_t* __restrict__ pcode,
                       const float* __restrict__ y, const double* __restrict__ s_in, double* __restrict__ h) {
    const double s = *s_in;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
        const int cnt = jcnt(pcode[i]);
        const double dinv = cnt ? dx2 / (double)cnt : 0.0;
        h[i] = dinv * f[i] + s * (double)y[i];
    }
}

// q = A h = -L h; partials <f,h>, <h,q>, <f,p> (slots 0, 1, 2 of part, MAX_BLOCKS apart)
__global__ void __launch_bounds__(NT) k_loss_dots(Geo g, const uint8_t* __restrict__ pcode, const double* __restrict__ f,
                                                  const double* __restrict__ p, const double* __restrict__ h,
                                                  double* __restrict__ q, double* __restrict__ part) {
    __shared__ double sh[12];
    const double idx2 = 1.0 / (g.dx * g.dx);
    const long long n = (long long)g.nx * g.ny * g.nz;
    double v[3] = {0.0, 0.0, 0.0};
    for (long long c = (long long)blockIdx.x * NT + threadIdx.x; c < n; c += (long long)gridDim.x * NT) {
        const int i = (int)(c % g.nx), j = (int)((c / g.nx) % g.ny), k = (int)(c / ((long long)g.nx * g.ny));
        const uint8_t pc = pcode[c];
        const double hc = h[c];
        double acc = (double)jcnt(pc) * hc;
        for (int d = 0; d < 6; ++d) {
            if (pc & (1 << d)) {
                bool bnd;
                acc -= h[nb_index(g, i, j, k, d, bnd)];
            }
        }
        const double qc = acc * idx2;
        q[c] = qc;
        v[0] += f[c] * hc;
        v[1] += hc * qc;
        v[2] += f[c] * p[c];
    }
    block_reduce<3>(v, sh);
    if (threadIdx.x == 0) {
        part[blockIdx.x] = v[0];
        part[MAX_BLOCKS + blockIdx.x] = v[1];
        part[2 * MAX_BLOCKS + blockIdx.x] = v[2];
    }
}

// loss = 1 - c^2 / (B Q); scal[1] = s 2c/(BQ), scal[2] = c/Q (gradient coefficients)
__global__ void __launch_bounds__(NT) k_loss_final(const double* __restrict__ part, int nparts, double* __restrict__ scal) {
    __shared__ double sh[12];
    double v[3] = {0.0, 0.0, 0.0};
    for (int b = threadIdx.x; b < nparts; b += NT) {
        v[0] += part[b];
        v[1] += part[MAX_BLOCKS + b];
        v[2] += part[2 * MAX_BLOCKS + b];
    }
    block_reduce<3>(v, sh);
    if (threadIdx.x == 0) {
        const double c = v[0], Q = v[1], B = v[2];
        const double s = scal[0];
        scal[3] = 1.0 - c * c / (B * Q);
        scal[1] = s * 2.0 * c / (B * Q);
        scal[2] = c / Q;
    }
}

// d loss / d y = s (2c/(BQ)) ((c/Q) q - f), rounded to BF16 for the backward pass
__global__ void k_dy(long long n, const double* __restrict__ q, const double* __restrict__ f,
                     const double* __restrict__ scal, uint16_t* __restrict__ dy) {
    const double k1 = scal[1], k2 = scal[2];
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        dy[i] = f2bf((float)(k1 * (k2 * q[i] - f[i])));
}

// --- the training loss through the smoothed preconditioner (S = omega D^-1) ---

// y = A x = -L x (double), one cell per thread
__global__ void __launch_bounds__(NT) k_amul(Geo g, const uint8_t* __restrict__ pcode, const double* __restrict__ x,
                                             double* __restrict__ y) {
    const double idx2 = 1.0 / (g.dx * g.dx);
    const long long n = (long long)g.nx * g.ny * g.nz;
    for (long long c = (long long)blockIdx.x * NT + threadIdx.x; c < n; c += (long long)gridDim.x * NT) {
        const int i = (int)(c % g.nx), j = (int)((c / g.nx) % g.ny), k = (int)(c / ((long long)g.nx * g.ny));
        const uint8_t pc = pcode[c];
        double acc = (double)jcnt(pc) * x[c];
        for (int d = 0; d < 6; ++d) {
            if (pc & (1 << d)) {
                bool bnd;
                acc -= x[nb_index(g, i, j, k, d, bnd)];
            }
        }
        y[c] = acc * idx2;
    }
}

// elementwise steps; out may be a, b or c (no restrict):
// SM_S: out = S a;  SM_SUB: out = a - b;  SM_POST: out = a + S (b - c)
enum { SM_S = 0, SM_SUB = 1, SM_POST = 2 };
__global__ void k_sm_step(long long n, int mode, double omega, double dx2, const uint8_t* __restrict__ pcode,
                          const double* a, const double* b, const double* c, double* out) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
        const int cnt = jcnt(pcode[i]);
        const double sw = cnt ? omega * dx2 / (double)cnt : 0.0;
        if (mode == SM_S)
            out[i] = sw * a[i];
        else if (mode == SM_SUB)
            out[i] = a[i] - b[i];
        else
            out[i] = a[i] + sw * (b[i] - c[i]);
    }
}

// z2 = t + D^-1 r1 + s y (out may be r1)
__global__ void k_z2(long long n, double dx2, const uint8_t* __restrict__ pcode, const double* t, const double* r1,
                     const float* __restrict__ y, const double* __restrict__ s_in, double* out) {
    const double s = *s_in;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
        const int cnt = jcnt(pcode[i]);
        const double dinv = cnt ? dx2 / (double)cnt : 0.0;
        out[i] = t[i] + dinv * r1[i] + s * (double)y[i];
    }
}

// G = s (2c/(BQ)) ((c/Q) q - f): the signal k_dy rounds, kept in double
__global__ void k_gph(long long n, const double* __restrict__ q, const double* __restrict__ f,
                      const double* __restrict__ scal, double* __restrict__ out) {
    const double k1 = scal[1], k2 = scal[2];
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        out[i] = k1 * (k2 * q[i] - f[i]);
}

// dy = BF16(a - b)
__global__ void k_dy_diff(long long n, const double* __restrict__ a, const double* __restrict__ b,
                          uint16_t* __restrict__ dy) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        dy[i] = f2bf((float)(a[i] - b[i]));
}

__global__ void k_neg(long long n, const double* __restrict__ a, double* __restrict__ b) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        b[i] = -a[i];
}

__global__ void k_f32_to_bf16(long long n, const float* __restrict__ a, uint16_t* __restrict__ b) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        b[i] = f2bf(a[i]);
}

// Adam (Kingma & Ba): step t >= 1, beta1 0.9, beta2 0.999, eps 1e-8
__global__ void k_adam(int n, float* __restrict__ w, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, int t, float lr) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float b1 = 0.9f, b2 = 0.999f;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float mh = mi / (1.0f - powf(b1, (float)t));
    const float vh = vi / (1.0f - powf(b2, (float)t));
    w[i] = w[i] - lr * mh / (sqrtf(vh) + 1e-8f);
}

}  // namespace

}  // namespace ibm

// ------------------------------------------------------------------ network object

struct ibm_cnn {
    int device;
    long long cap;
    float* w;        // FP32 master weights (flat, ABI layout)
    float* m;        // Adam moments
    float* v;
    float* dw;       // last gradient
    int adam_t;
    uint16_t* wp;    // packed BF16 A operands of the six convolutions
    ibm::PackDesc pd[7];
    uint16_t* xr;    // network input (residual / s), cells
    uint16_t* xg;    // geometry input, cells
    uint16_t* G;     // gate, cells x 16
    uint16_t* u1;    // W1 * x before the gate (training), cells x 16
    uint16_t* a1;    // (W1 * x) . G
    uint16_t* y;     // W2 * a1
    uint16_t* vv;    // W2^T * y before the gate (training)
    uint16_t* bb;    // (W2^T * y) . G
    uint16_t* sig[2];// backward signals, cells x 16
    uint16_t* dy1;   // BF16 output gradient, cells
    float* dG;       // gate gradient, cells x 16
    float* out;      // K^T K x, cells
    float* wpart;    // WG_MAX_BLOCKS x 27 x 256
    double* h;       // cap (loss)
    double* q;       // cap
    double* f;       // cap (loss: -b)
    double* part;    // 3 x MAX_BLOCKS
    double* cpart;   // 2 x (blocks of the marching kernels of the attached geometry)
    long long cpart_n;
    double* scal;    // 8: s, k1, k2, loss
    double* h_scal;  // pinned host copy
    int nx, ny, nz;  // dims of the last forward
    bool have_fwd;
    bool train_ok;   // training buffers allocated (not IBM_CNN_INFERENCE_ONLY)
};

namespace ibm {
namespace {

enum { PV_W1 = 0, PV_W2, PV_W2T, PV_W1T, PV_WG, PV_WGT, PV_W1TY, PV_N };
constexpr int OFF_W1 = 0, OFF_W2 = 432, OFF_WG = 7344;

void fill_pack_desc(ibm_cnn* n) {
    // (layer offset, layer cin, layer cout, adjoint, dy rows)
    const int spec[PV_N][5] = {{OFF_W1, 1, 16, 0, 0}, {OFF_W2, 16, 16, 0, 0}, {OFF_W2, 16, 16, 1, 0},
                               {OFF_W1, 1, 16, 1, 0}, {OFF_WG, 1, 16, 0, 0}, {OFF_WG, 1, 16, 1, 0},
                               {OFF_W1, 1, 16, 1, 1}};
    int off = 0;
    for (int v = 0; v < PV_N; ++v) {
        PackDesc d;
        d.loff = spec[v][0];
        d.lcin = spec[v][1];
        d.lcout = spec[v][2];
        d.bwd = spec[v][3];
        d.ymode = spec[v][4];
        d.cin = d.bwd ? d.lcout : d.lcin;
        d.cout = d.bwd ? d.lcin : d.lcout;
        d.ks = d.ymode ? 5 : ksteps(d.cin);
        d.off = off;
        off += d.ks * 512;
        n->pd[v] = d;
    }
}

int packed_elems(const ibm_cnn* n) { return n->pd[PV_N - 1].off + n->pd[PV_N - 1].ks * 512; }

int repack(ibm_cnn* n, hipStream_t s) {
    for (int v = 0; v < PV_N; ++v) {
        const int tot = n->pd[v].ks * 512;
        k_pack<<<(tot + 255) / 256, 256, 0, s>>>(n->w, n->wp, n->pd[v]);
    }
    IBM_HIP(hipGetLastError());
    return IBM_OK;
}

int conv_blocks(int nx, int ny, int nz) {
    return ((nx + CTX - 1) / CTX) * ((ny + CTY - 1) / CTY) * ((nz + CTZ - 1) / CTZ);
}

const uint16_t* pw(const ibm_cnn* n, int v) { return n->wp + n->pd[v].off; }

ConvIO io_none(int ostride = 1) { return ConvIO{nullptr, nullptr, nullptr, nullptr, 0, ostride}; }
ConvIO io_gate(const uint16_t* G, uint16_t* aux) { return ConvIO{G, aux, nullptr, nullptr, 0, 1}; }
ConvIO io_bgate(const uint16_t* G, const uint16_t* pre, float* dg, int accum) {
    return ConvIO{G, nullptr, pre, dg, accum, 1};
}

// G = hsig(Wg * xg)
int net_gate(ibm_cnn* n, int nx, int ny, int nz, hipStream_t s) {
    k_conv<1, 16, EPI_HSIG><<<conv_blocks(nx, ny, nz), 256, 0, s>>>(nx, ny, nz, n->xg, pw(n, PV_WG), n->G,
                                                                        io_none(), nullptr, 0);
    IBM_HIP(hipGetLastError());
    return IBM_OK;
}

// out = K^T K xr with the current gate; `keep` stores the pre-gate activations for
// the backward pass
// Concurrent blocks of the marching kernels on the current device: three per CU (their
// LDS, 45 to 52 KB per block, and registers, at most 168 VGPRs, are sized for that).
int mconv_slots() {
    static int cached[64] = {0};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) dev = 0;
    if (!cached[dev]) {
        int ncu = 0;
        if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || ncu <= 0)
            ncu = 256;
        cached[dev] = 3 * ncu;
    }
    return cached[dev];
}

// Planes per slab of the march.  A block costs (its planes + 3 prologue planes) plane
// steps and all block slots run at about the same pace, so the march takes
// (waves of blocks) x (planes per slab + 3); the slab count minimising that is taken
// (the fewest slabs among equals).  256^3 on 256 CUs: 3 slabs of 86 planes, 768 blocks
// in one wave (8 slabs of 32 planes took 2.67 waves).
int mconv_planes(int nx, int ny, int nz) {
    const long long txy = (long long)((nx + CTX - 1) / CTX) * ((ny + CTY - 1) / CTY);
    const long long slots = mconv_slots();
    long long best = -1;
    int best_mz = nz;
    for (int S = 1; S <= nz; ++S) {
        const int mz = (nz + S - 1) / S;
        if ((nz + mz - 1) / mz != S) continue;   // the same slabs as a smaller count
        const long long cost = ((txy * S + slots - 1) / slots) * (mz + 3);
        if (best < 0 || cost < best) {
            best = cost;
            best_mz = mz;
        }
    }
    return best_mz;
}

int mconv_blocks(int nx, int ny, int nz, int mz) {
    return ((nx + CTX - 1) / CTX) * ((ny + CTY - 1) / CTY) * ((nz + mz - 1) / mz);
}

int net_forward(ibm_cnn* n, int nx, int ny, int nz, bool keep, hipStream_t s) {
    if (!keep) {
        // solver path: marching kernels, no activations kept (their in-plane byte
        // offsets are 32-bit)
        if ((long long)nx * ny * 32 >= (1LL << 31)) {
            set_error("cnn: x-y plane too large for the marching convolutions");
            return IBM_ERR_ARG;
        }
        const int mz = mconv_planes(nx, ny, nz);
        const int mb = mconv_blocks(nx, ny, nz, mz);
        const uint16_t* wg = pw(n, PV_WG);
        k_mfwd<false><<<mb, 256, 0, s>>>(nx, ny, nz, mz, n->xr, n->xg, pw(n, PV_W1), wg, pw(n, PV_W2), n->y,
                                         nullptr, 0, nullptr, nullptr, 0);
        // the gated adjoint output goes to a1's buffer (the forward half keeps a1 in LDS)
        k_mconv<16, EPI_GATE><<<mb, 256, 0, s>>>(nx, ny, nz, mz, n->y, pw(n, PV_W2T), n->a1, n->xg, wg, nullptr,
                                                     0, CombineIO{});
        k_mconv<1, EPI_F32><<<mb, 256, 0, s>>>(nx, ny, nz, mz, n->a1, pw(n, PV_W1TY), n->out, nullptr, nullptr,
                                                   nullptr, 0, CombineIO{});
        IBM_HIP(hipGetLastError());
        n->nx = nx;
        n->ny = ny;
        n->nz = nz;
        n->have_fwd = false;
        return IBM_OK;
    }
    const int nb = conv_blocks(nx, ny, nz);
    k_conv<1, 16, EPI_GATE><<<nb, 256, 0, s>>>(nx, ny, nz, n->xr, pw(n, PV_W1), n->a1,
                                               io_gate(n->G, keep ? n->u1 : nullptr), nullptr, 0);
    k_conv<16, 16, EPI_BF16><<<nb, 256, 0, s>>>(nx, ny, nz, n->a1, pw(n, PV_W2), n->y, io_none(), nullptr, 0);
    k_conv<16, 16, EPI_GATE><<<nb, 256, 0, s>>>(nx, ny, nz, n->y, pw(n, PV_W2T), n->bb,
                                                io_gate(n->G, keep ? n->vv : nullptr), nullptr, 0);
    k_conv<16, 1, EPI_F32><<<nb, 256, 0, s>>>(nx, ny, nz, n->bb, pw(n, PV_W1T), n->out, io_none(1), nullptr, 0);
    IBM_HIP(hipGetLastError());
    n->nx = nx;
    n->ny = ny;
    n->nz = nz;
    n->have_fwd = keep;
    return IBM_OK;
}

template <int CIN, int COUT>
int wgrad(ibm_cnn* n, const uint16_t* x, const uint16_t* dy, int off, int accum, hipStream_t s) {
    const int nx = n->nx, ny = n->ny, nz = n->nz;
    const int ntiles = conv_blocks(nx, ny, nz);
    const int nb = ntiles < WG_MAX_BLOCKS ? ntiles : WG_MAX_BLOCKS;
    k_wgrad<CIN, COUT><<<nb, 256, 0, s>>>(nx, ny, nz, x, dy, n->wpart, ntiles);
    const int nw = 27 * CIN * COUT;
    k_wsum<<<(nw + 255) / 256, 256, 0, s>>>(n->wpart, nb, CIN, COUT, n->dw + off, accum);
    IBM_HIP(hipGetLastError());
    return IBM_OK;
}

// Backward pass of the kept forward for d J / d out = dy1 (BF16): dW into n->dw; when
// dx is non-null, dJ/dxr and dJ/dxg into dx (cells x 2 floats).
int net_backward(ibm_cnn* n, float* dx, hipStream_t s) {
    const int nx = n->nx, ny = n->ny, nz = n->nz;
    const int nb = conv_blocks(nx, ny, nz);
    const long long cells = (long long)nx * ny * nz;
    int rc;
    // out = W1^T * bb
    if ((rc = wgrad<1, 16>(n, n->dy1, n->bb, OFF_W1, 0, s))) return rc;
    // d bb = W1 * dy1;  d vv = d bb . G;  dG = d bb . vv
    k_conv<1, 16, EPI_BGATE><<<nb, 256, 0, s>>>(nx, ny, nz, n->dy1, pw(n, PV_W1), n->sig[0],
                                                io_bgate(n->G, n->vv, n->dG, 0), nullptr, 0);
    // vv = W2^T * y
    if ((rc = wgrad<16, 16>(n, n->sig[0], n->y, OFF_W2, 0, s))) return rc;
    // d y = W2 * d vv
    k_conv<16, 16, EPI_BF16><<<nb, 256, 0, s>>>(nx, ny, nz, n->sig[0], pw(n, PV_W2), n->sig[1], io_none(), nullptr, 0);
    // y = W2 * a1
    if ((rc = wgrad<16, 16>(n, n->a1, n->sig[1], OFF_W2, 1, s))) return rc;
    // d a1 = W2^T * d y;  d u1 = d a1 . G;  dG += d a1 . u1
    k_conv<16, 16, EPI_BGATE><<<nb, 256, 0, s>>>(nx, ny, nz, n->sig[1], pw(n, PV_W2T), n->sig[0],
                                                 io_bgate(n->G, n->u1, n->dG, 1), nullptr, 0);
    // u1 = W1 * xr
    if ((rc = wgrad<1, 16>(n, n->xr, n->sig[0], OFF_W1, 1, s))) return rc;
    if (dx)
        k_conv<16, 1, EPI_F32><<<nb, 256, 0, s>>>(nx, ny, nz, n->sig[0], pw(n, PV_W1T), dx, io_none(2), nullptr, 0);
    // G = hsig(Wg * xg)
    k_dpre<<<2048, 256, 0, s>>>(cells * 16, n->dG, n->G, n->sig[1]);
    if ((rc = wgrad<1, 16>(n, n->xg, n->sig[1], OFF_WG, 0, s))) return rc;
    if (dx)
        k_conv<16, 1, EPI_F32><<<nb, 256, 0, s>>>(nx, ny, nz, n->sig[1], pw(n, PV_WGT), dx + 1, io_none(2), nullptr, 0);
    IBM_HIP(hipGetLastError());
    return IBM_OK;
}

int check_grid(const ibm_cnn* n, long long cells) {
    if (cells <= 0 || cells > n->cap) {
        set_error("cnn: grid has more cells than the network was created for");
        return IBM_ERR_ARG;
    }
    return IBM_OK;
}

// geometry input of the context (and, for training networks, the stored gate the
// training kernels use; the solver path computes the gate on the fly)
// Block partials of the combine epilogue for the context's grid: two sums per block of
// the marching launch.  Grow-only; sized by ibm_ctx_set_preconditioner (set-up), and by
// the stand-alone network calls, never inside a solve.
int size_partials(ibm_cnn* n, const Geo& g, hipStream_t s) {
    const long long need = 2LL * mconv_blocks(g.nx, g.ny, g.nz, mconv_planes(g.nx, g.ny, g.nz));
    if (n->cpart_n >= need) return IBM_OK;
    IBM_HIP(hipStreamSynchronize(s));
    if (n->cpart) IBM_HIP(hipFree(n->cpart));
    n->cpart = nullptr;
    n->cpart_n = 0;
    IBM_HIP(ibm::dev_malloc((void**)&n->cpart, need * sizeof(double)));
    n->cpart_n = need;
    return IBM_OK;
}

// Geometry channel (and, for a trainable network, its gate) of the context's grid.
// Allocates nothing: the partials must already be sized for this grid.
int prepare_geometry(ibm_cnn* n, ibm_ctx* c, hipStream_t s) {
    const Geo& g = c->geo;
    const long long need = 2LL * mconv_blocks(g.nx, g.ny, g.nz, mconv_planes(g.nx, g.ny, g.nz));
    if (n->cpart_n < need) {
        set_error("cnn: network not prepared for this grid (attach it with ibm_ctx_set_preconditioner)");
        return IBM_ERR_ARG;
    }
    k_geom<<<2048, 256, 0, s>>>(c->N, c->pcode, n->xg);
    IBM_HIP(hipGetLastError());
    return n->train_ok ? net_gate(n, c->geo.nx, c->geo.ny, c->geo.nz, s) : IBM_OK;
}

int need_training(const ibm_cnn* n, const char* what) {
    if (!n->train_ok) {
        set_error(std::string(what) + ": network was created inference-only");
        return IBM_ERR_ARG;
    }
    return IBM_OK;
}

// Loss of one pair (b, p), L p = b, on the context's stencil, and the gradient signal
// d loss / d out in dy1 (BF16): f = -b, s = RMS(f), h = D^-1 f + s K^T K (f/s),
// loss = 1 - (f.h)^2 / ((f.p)(h.A h)).  scal[3] = loss.
// omega > 0: h is the smoothed form (S = omega D^-1): t = S f, r1 = f - A t, s = RMS(r1),
// z2 = t + D^-1 r1 + s K^T K (r1/s), h = z2 + S (f - A z2), and the signal reaching the
// network's output is (I - A S) applied to the unsmoothed one.  Buffers: f; q holds t,
// then A z2, A h, S G; h holds A t, r1, z2, h, then G; f finally holds A S G.
int loss_forward(ibm_cnn* n, ibm_ctx* c, const double* b, const double* p, double omega, hipStream_t s) {
    const Geo& g = c->geo;
    const long long N = c->N;
    const int nred = 1024;
    const double dx2 = g.dx * g.dx;
    int rc = size_partials(n, g, s);
    if (!rc) rc = prepare_geometry(n, c, s);
    if (rc) return rc;
    const bool smooth = omega > 0.0;
    k_neg<<<2048, 256, 0, s>>>(N, b, n->f);
    const double* rin = n->f;
    if (smooth) {
        k_sm_step<<<2048, 256, 0, s>>>(N, SM_S, omega, dx2, c->pcode, n->f, nullptr, nullptr, n->q);
        k_amul<<<nred, NT, 0, s>>>(g, c->pcode, n->q, n->h);
        k_sm_step<<<2048, 256, 0, s>>>(N, SM_SUB, omega, dx2, c->pcode, n->f, n->h, nullptr, n->h);
        rin = n->h;
    }
    k_sumsq<double><<<nred, NT, 0, s>>>(N, rin, n->part);
    k_input<double><<<nred, NT, 0, s>>>(N, rin, n->part, nred, n->xr, n->scal, nullptr, 0, 0);
    IBM_HIP(hipGetLastError());
    if ((rc = net_forward(n, g.nx, g.ny, g.nz, true, s))) return rc;
    if (smooth) {
        k_z2<<<2048, 256, 0, s>>>(N, dx2, c->pcode, n->q, n->h, n->out, n->scal, n->h);
        k_amul<<<nred, NT, 0, s>>>(g, c->pcode, n->h, n->q);
        k_sm_step<<<2048, 256, 0, s>>>(N, SM_POST, omega, dx2, c->pcode, n->h, n->f, n->q, n->h);
    } else {
        k_phat<<<2048, 256, 0, s>>>(N, dx2, n->f, c->pcode, n->out, n->scal, n->h);
    }
    k_loss_dots<<<nred, NT, 0, s>>>(g, c->pcode, n->f, p, n->h, n->q, n->part);
    k_loss_final<<<1, NT, 0, s>>>(n->part, nred, n->scal);
    if (smooth) {
        k_gph<<<2048, 256, 0, s>>>(N, n->q, n->f, n->scal, n->h);
        k_sm_step<<<2048, 256, 0, s>>>(N, SM_S, omega, dx2, c->pcode, n->h, nullptr, nullptr, n->q);
        k_amul<<<nred, NT, 0, s>>>(g, c->pcode, n->q, n->f);
        k_dy_diff<<<2048, 256, 0, s>>>(N, n->h, n->f, n->dy1);
    } else {
        k_dy<<<2048, 256, 0, s>>>(N, n->q, n->f, n->scal, n->dy1);
    }
    IBM_HIP(hipGetLastError());
    return IBM_OK;
}

}  // namespace

// Gate of the context's geometry; called once per solve before the FCG segments.
int cnn_prepare_geometry(void* net, ibm_ctx* c, hipStream_t s) {
    return prepare_geometry(static_cast<ibm_cnn*>(net), c, s);
}

// z = D^-1 r + s K^T K (r/s) inside the FCG solve (see poisson.hip): s^2 = <r,r>/N from
// the partials in rr_slot; <z,r> -> zr_slot, <z,rp> -> zrp_slot (-1: none).  With check,
// stops the solve at iteration it (converged = 1) when <r,r> <= sv->tol2.  The gate must be
// prepared.
// omega > 0: the symmetric two-level form with S = omega D^-1: r1 = r - A S r (into the
// network's FP32 output buffer, <r1,r1> partials in r1_slot), the network on r1, then
// z2 = S r + D^-1 r1 + s K^T K (r1/s) from the combine epilogue (into the 16-channel
// buffer y, free once the gated adjoint has read it) and z = z2 + S (r - A z2) with the
// dot products; nx % 4 == 0.
int cnn_precondition_solver(void* net, ibm_ctx* c, const float* r, const float* rp, float* z, double* partials,
                            int nparts, int rr_slot, int zr_slot, int zrp_slot, int r1_slot, double omega, Solver* sv,
                            int it, int check, hipStream_t s) {
    ibm_cnn* n = static_cast<ibm_cnn*>(net);
    const Geo& g = c->geo;
    const int nx = g.nx, ny = g.ny, nz = g.nz;
    if ((long long)nx * ny * 32 >= (1LL << 31)) {
        set_error("cnn: x-y plane too large for the marching convolutions");
        return IBM_ERR_ARG;
    }
    const bool smooth = omega > 0.0;
    if (smooth && (nx % 4 != 0 || (uintptr_t)r % 16 || (uintptr_t)z % 16 || (uintptr_t)rp % 16)) {
        set_error("cnn: the smoothed preconditioner needs nx % 4 == 0 and 16-byte aligned vectors");
        return IBM_ERR_ARG;
    }
    const int mz = mconv_planes(nx, ny, nz);
    const int mb = mconv_blocks(nx, ny, nz, mz);
    if (2LL * mb > n->cpart_n) {
        set_error("cnn: geometry not prepared for this network");
        return IBM_ERR_ARG;
    }
    const uint16_t* wg = pw(n, PV_WG);
    const double* rpart = partials + (long long)rr_slot * MAX_BLOCKS;
    // kernels after the stop test of iteration it (k_input's, or the pre-smoothing's) run
    // only while the solve goes on past it; without that test (the fused FCG tests in its
    // pass A, after these) they run up to and including iteration it
    const int gate = check ? it + 1 : it;
    const float* rin = r;
    if (smooth) {
        int rc = smooth_pre(c, r, n->out, omega, partials, nparts, r1_slot, rr_slot, sv, it, check, s);
        if (rc) return rc;
        rin = n->out;
        rpart = partials + (long long)r1_slot * MAX_BLOCKS;
    }
    if (smooth && sv) {
        launch_timed(c, TK_DIR, k_mfwd<true>, mb, s, nx, ny, nz, mz, (const void*)rin, (const uint16_t*)n->xg,
                     pw(n, PV_W1), wg, pw(n, PV_W2), n->y, rpart, nparts, n->scal, (const Solver*)sv, gate);
    } else if (smooth) {
        k_mfwd<true><<<mb, 256, 0, s>>>(nx, ny, nz, mz, rin, n->xg, pw(n, PV_W1), wg, pw(n, PV_W2), n->y, rpart,
                                        nparts, n->scal, sv, gate);
    } else if (check) {
        // k_input also stops the solve once <r,r> <= tol^2 |b|^2
        k_input<float><<<nparts, NT, 0, s>>>(c->N, r, rpart, nparts, n->xr, n->scal, sv, it, check);
        k_mfwd<false><<<mb, 256, 0, s>>>(nx, ny, nz, mz, n->xr, n->xg, pw(n, PV_W1), wg, pw(n, PV_W2), n->y,
                                         nullptr, 0, nullptr, sv, gate);
    } else if (sv) {   // inside a solve: the dominant kernel is timed when the context times its kernels
        launch_timed(c, TK_DIR, k_mfwd<true>, mb, s, nx, ny, nz, mz, (const void*)r, (const uint16_t*)n->xg,
                     pw(n, PV_W1), wg, pw(n, PV_W2), n->y, rpart, nparts, n->scal, (const Solver*)sv, gate);
    } else {
        k_mfwd<true><<<mb, 256, 0, s>>>(nx, ny, nz, mz, r, n->xg, pw(n, PV_W1), wg, pw(n, PV_W2), n->y, rpart,
                                        nparts, n->scal, sv, gate);
    }
    k_mconv<16, EPI_GATE><<<mb, 256, 0, s>>>(nx, ny, nz, mz, n->y, pw(n, PV_W2T), n->a1, n->xg, wg, sv, gate,
                                                 CombineIO{});
    if (smooth) {
        float* z2 = reinterpret_cast<float*>(n->y);
        const CombineIO cio{rin, r, c->pcode, n->scal, g.dx * g.dx, z2, n->cpart, (float)omega};
        k_mconv<1, EPI_COMBINE><<<mb, 256, 0, s>>>(nx, ny, nz, mz, n->a1, pw(n, PV_W1TY), nullptr, nullptr,
                                                       nullptr, sv, gate, cio);
        IBM_HIP(hipGetLastError());
        int rc = smooth_post(c, z2, r, rp, z, omega, partials, nparts, zr_slot, zrp_slot, sv, gate, s);
        if (rc) return rc;
    } else {
        const CombineIO cio{r, rp, c->pcode, n->scal, g.dx * g.dx, z, n->cpart};
        k_mconv<1, EPI_COMBINE><<<mb, 256, 0, s>>>(nx, ny, nz, mz, n->a1, pw(n, PV_W1TY), nullptr, nullptr,
                                                       nullptr, sv, gate, cio);
        k_relay<<<1, NT, 0, s>>>(n->cpart, mb, partials, nparts, zr_slot, zrp_slot, sv, gate);
    }
    IBM_HIP(hipGetLastError());
    n->nx = nx;
    n->ny = ny;
    n->nz = nz;
    n->have_fwd = false;
    return IBM_OK;
}

bool cnn_covers(const void* net, long long cells) { return net && static_cast<const ibm_cnn*>(net)->cap >= cells; }

}  // namespace ibm

// ------------------------------------------------------------------ C ABI

using namespace ibm;

namespace {

void net_free(ibm_cnn* n) {
    if (!n) return;
    void* bufs[] = {n->w,  n->m,  n->v,      n->dw,     n->wp,  n->xr,    n->xg,  n->G, n->u1, n->a1, n->y,
                    n->vv, n->bb, n->sig[0], n->sig[1], n->dy1, n->dG,    n->out, n->wpart, n->h, n->q,  n->f,
                    n->part, n->cpart, n->scal};
    for (void* b : bufs)
        if (b) (void)hipFree(b);
    if (n->h_scal) (void)hipHostFree(n->h_scal);
    delete n;
}

int net_check(const ibm_cnn* n) {
    if (!n) {
        set_error("cnn: null network");
        return IBM_ERR_ARG;
    }
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != n->device) {
        set_error("cnn: call on a device other than the one the network was created on");
        return IBM_ERR_ARG;
    }
    return IBM_OK;
}

}  // namespace

extern "C" {

int ibm_cnn_create(int64_t max_cells, int32_t flags, ibm_cnn** out) try {
    if (!out || max_cells <= 0 || (flags & ~IBM_CNN_INFERENCE_ONLY)) {
        set_error("ibm_cnn_create: bad arguments");
        return IBM_ERR_ARG;
    }
    *out = nullptr;
    ibm_cnn* n = new (std::nothrow) ibm_cnn();
    if (!n) {
        set_error("ibm_cnn_create: host allocation failed");
        return IBM_ERR_OOM;
    }
    std::memset(n, 0, sizeof(*n));
    if (hipGetDevice(&n->device) != hipSuccess) {
        delete n;
        set_error("ibm_cnn_create: no HIP device");
        return IBM_ERR_HIP;
    }
    n->cap = max_cells;
    n->train_ok = !(flags & IBM_CNN_INFERENCE_ONLY);
    fill_pack_desc(n);
    const size_t cap = (size_t)max_cells;
    bool ok = true;
    auto alloc = [&](void** p, size_t bytes) {
        if (ok && ibm::dev_malloc(p, bytes) != hipSuccess) ok = false;
    };
    alloc((void**)&n->w, NWTS * sizeof(float));
    alloc((void**)&n->m, NWTS * sizeof(float));
    alloc((void**)&n->v, NWTS * sizeof(float));
    alloc((void**)&n->dw, NWTS * sizeof(float));
    alloc((void**)&n->wp, (size_t)packed_elems(n) * sizeof(uint16_t));
    alloc((void**)&n->xr, cap * sizeof(uint16_t));
    alloc((void**)&n->xg, cap * sizeof(uint16_t));
    alloc((void**)&n->a1, cap * 16 * sizeof(uint16_t));
    alloc((void**)&n->y, cap * 16 * sizeof(uint16_t));
    alloc((void**)&n->out, cap * sizeof(float));
    alloc((void**)&n->part, 3 * MAX_BLOCKS * sizeof(double));
    alloc((void**)&n->scal, 8 * sizeof(double));
    if (n->train_ok) {
        uint16_t** c16[] = {&n->G, &n->u1, &n->vv, &n->bb, &n->sig[0], &n->sig[1]};
        for (uint16_t** pp : c16) alloc((void**)pp, cap * 16 * sizeof(uint16_t));
        alloc((void**)&n->dy1, cap * sizeof(uint16_t));
        alloc((void**)&n->dG, cap * 16 * sizeof(float));
        alloc((void**)&n->wpart, (size_t)WG_MAX_BLOCKS * 27 * 256 * sizeof(float));
        alloc((void**)&n->h, cap * sizeof(double));
        alloc((void**)&n->q, cap * sizeof(double));
        alloc((void**)&n->f, cap * sizeof(double));
    }
    if (ok && ibm::host_malloc(&n->h_scal, 8 * sizeof(double)) != hipSuccess) ok = false;
    if (!ok) {
        net_free(n);
        set_error("ibm_cnn_create: device allocation failed");
        return IBM_ERR_OOM;
    }
    ok = hipMemset(n->w, 0, NWTS * sizeof(float)) == hipSuccess &&
         hipMemset(n->m, 0, NWTS * sizeof(float)) == hipSuccess &&
         hipMemset(n->v, 0, NWTS * sizeof(float)) == hipSuccess &&
         hipMemset(n->scal, 0, 8 * sizeof(double)) == hipSuccess;
    if (!ok || repack(n, nullptr) != IBM_OK || hipDeviceSynchronize() != hipSuccess) {
        net_free(n);
        set_error("ibm_cnn_create: initialisation failed");
        return IBM_ERR_HIP;
    }
    *out = n;
    return IBM_OK;
} IBM_CATCH_ALL

int ibm_cnn_destroy(ibm_cnn* net) try {
    if (!net) return IBM_OK;
    (void)hipDeviceSynchronize();
    net_free(net);
    return IBM_OK;
} IBM_CATCH_ALL

int ibm_cnn_set_weights(ibm_cnn* net, const float* w_host, int64_t n) try {
    int rc = net_check(net);
    if (rc) return rc;
    if (!w_host || n != NWTS) {
        set_error("ibm_cnn_set_weights: expected IBM_CNN_NWEIGHTS host floats");
        return IBM_ERR_ARG;
    }
    IBM_HIP(hipMemcpy(net->w, w_host, NWTS * sizeof(float), hipMemcpyHostToDevice));
    IBM_HIP(hipMemset(net->m, 0, NWTS * sizeof(float)));
    IBM_HIP(hipMemset(net->v, 0, NWTS * sizeof(float)));
    net->adam_t = 0;
    rc = repack(net, nullptr);
    if (rc) return rc;
    IBM_HIP(hipDeviceSynchronize());
    return IBM_OK;
} IBM_CATCH_ALL

int ibm_cnn_get_weights(ibm_cnn* net, float* w_host, int64_t n) try {
    int rc = net_check(net);
    if (rc) return rc;
    if (!w_host || n != NWTS) {
        set_error("ibm_cnn_get_weights: expected IBM_CNN_NWEIGHTS host floats");
        return IBM_ERR_ARG;
    }
    IBM_HIP(hipDeviceSynchronize());
    IBM_HIP(hipMemcpy(w_host, net->w, NWTS * sizeof(float), hipMemcpyDeviceToHost));
    return IBM_OK;
} IBM_CATCH_ALL

int ibm_cnn_forward(ibm_cnn* net, const uint16_t* x_dev, float* y_dev, int32_t nx, int32_t ny, int32_t nz,
                    void* stream) try {
    int rc = net_check(net);
    if (rc) return rc;
    if (!x_dev || !y_dev || nx <= 0 || ny <= 0 || nz <= 0) {
        set_error("ibm_cnn_forward: bad arguments");
        return IBM_ERR_ARG;
    }
    const long long cells = (long long)nx * ny * nz;
    if ((rc = check_grid(net, cells))) return rc;
    hipStream_t s = (hipStream_t)stream;
    k_split<<<2048, 256, 0, s>>>(cells, x_dev, net->xr, net->xg);
    IBM_HIP(hipGetLastError());
    if (net->train_ok) {
        if ((rc = net_gate(net, nx, ny, nz, s))) return rc;
        if ((rc = net_forward(net, nx, ny, nz, true, s))) return rc;
    } else if ((rc = net_forward(net, nx, ny, nz, false, s))) {
        return rc;
    }
    IBM_HIP(hipMemcpyAsync(y_dev, net->out, cells * sizeof(float), hipMemcpyDeviceToDevice, s));
    return IBM_OK;
} IBM_CATCH_ALL

int ibm_cnn_backward(ibm_cnn* net, const float* dy_dev, float* dw_dev, float* dx_dev, void* stream) try {
    int rc = net_check(net);
    if (rc) return rc;
    if ((rc = need_training(net, "ibm_cnn_backward"))) return rc;
    if (!dy_dev || !dw_dev) {
        set_error("ibm_cnn_backward: bad arguments");
        return IBM_ERR_ARG;
    }
    if (!net->have_fwd) {
        set_error("ibm_cnn_backward: no kept forward pass to differentiate");
        return IBM_ERR_ARG;
    }
    hipStream_t s = (hipStream_t)stream;
    const long long cells = (long long)net->nx * net->ny * net->nz;
    k_f32_to_bf16<<<2048, 256, 0, s>>>(cells, dy_dev, net->dy1);
    IBM_HIP(hipGetLastError());
    if ((rc = net_backward(net, dx_dev, s))) return rc;
    IBM_HIP(hipMemcpyAsync(dw_dev, net->dw, NWTS * sizeof(float), hipMemcpyDeviceToDevice, s));
    return IBM_OK;
} IBM_CATCH_ALL

int ibm_cnn_loss(ibm_cnn* net, ibm_ctx* ctx, const double* b_dev, const double* p_dev, double omega,
                 double* loss_out, float* dw_dev, void* stream) try {
    int rc = net_check(net);
    if (rc) return rc;
    if ((rc = need_training(net, "ibm_cnn_loss"))) return rc;
    if (!ctx || !ctx->stencil_ready || !b_dev || !p_dev || !(omega >= 0.0 && omega <= 1.0)) {
        set_error("ibm_cnn_loss: bad arguments (context needs a stencil, omega in [0, 1])");
        return IBM_ERR_ARG;
    }
    if ((rc = check_grid(net, ctx->N))) return rc;
    hipStream_t s = (hipStream_t)stream;
    if ((rc = loss_forward(net, ctx, b_dev, p_dev, omega, s))) return rc;
    if (dw_dev) {
        if ((rc = net_backward(net, nullptr, s))) return rc;
        IBM_HIP(hipMemcpyAsync(dw_dev, net->dw, NWTS * sizeof(float), hipMemcpyDeviceToDevice, s));
    }
    IBM_HIP(hipMemcpyAsync(net->h_scal, net->scal, 8 * sizeof(double), hipMemcpyDeviceToHost, s));
    IBM_HIP(hipStreamSynchronize(s));
    if (loss_out) *loss_out = net->h_scal[3];
    return IBM_OK;
} IBM_CATCH_ALL

int ibm_cnn_train_step(ibm_cnn* net, ibm_ctx* ctx, const double* b_dev, const double* p_dev, float lr,
                       double omega, double* loss_out, void* stream) try {
    int rc = net_check(net);
    if (rc) return rc;
    if ((rc = need_training(net, "ibm_cnn_train_step"))) return rc;
    if (!ctx || !ctx->stencil_ready || !b_dev || !p_dev || !(lr > 0.0f) || !(omega >= 0.0 && omega <= 1.0)) {
        set_error("ibm_cnn_train_step: bad arguments (context needs a stencil, lr > 0, omega in [0, 1])");
        return IBM_ERR_ARG;
    }
    if ((rc = check_grid(net, ctx->N))) return rc;
    hipStream_t s = (hipStream_t)stream;
    if ((rc = loss_forward(net, ctx, b_dev, p_dev, omega, s))) return rc;
    if ((rc = net_backward(net, nullptr, s))) return rc;
    net->adam_t += 1;
    k_adam<<<(NWTS + 255) / 256, 256, 0, s>>>(NWTS, net->w, net->dw, net->m, net->v, net->adam_t, lr);
    IBM_HIP(hipGetLastError());
    if ((rc = repack(net, s))) return rc;
    IBM_HIP(hipMemcpyAsync(net->h_scal, net->scal, 8 * sizeof(double), hipMemcpyDeviceToHost, s));
    IBM_HIP(hipStreamSynchronize(s));
    if (loss_out) *loss_out = net->h_scal[3];
    return IBM_OK;
} IBM_CATCH_ALL

int ibm_cnn_precondition(ibm_cnn* net, ibm_ctx* ctx, const float* r_dev, float* z_dev, double omega,
                         void* stream) try {
    int rc = net_check(net);
    if (rc) return rc;
    if (!ctx || !ctx->stencil_ready || !r_dev || !z_dev) {
        set_error("ibm_cnn_precondition: bad arguments (context needs a stencil)");
        return IBM_ERR_ARG;
    }
    if ((rc = check_grid(net, ctx->N))) return rc;
    if (!(omega >= 0.0 && omega <= 1.0)) {
        set_error("ibm_cnn_precondition: omega must lie in [0, 1]");
        return IBM_ERR_ARG;
    }
    hipStream_t s = (hipStream_t)stream;
    const int nred = 1024;
    if ((rc = size_partials(net, ctx->geo, s))) return rc;
    if ((rc = prepare_geometry(net, ctx, s))) return rc;
    k_sumsq<float><<<nred, NT, 0, s>>>(ctx->N, r_dev, net->part);
    IBM_HIP(hipGetLastError());
    // partial slot 0 of net->part holds <r,r>; <z,r> goes to slot 1, <r1,r1> of the
    // smoothed form to slot 2
    return cnn_precondition_solver(net, ctx, r_dev, nullptr, z_dev, net->part, nred, 0, 1, -1, 2, omega, nullptr, 0,
                                   0, s);
} IBM_CATCH_ALL

int ibm_ctx_set_preconditioner(ibm_ctx* ctx, ibm_cnn* net) try {
    if (!ctx) {
        set_error("ibm_ctx_set_preconditioner: null context");
        return IBM_ERR_ARG;
    }
    if (net) {
        int rc = net_check(net);
        if (rc) return rc;
        if (net->cap < ctx->N) {
            set_error("ibm_ctx_set_preconditioner: network workspace smaller than the grid");
            return IBM_ERR_ARG;
        }
        // set-up: size the network's partials for this grid so the solves never allocate
        if ((rc = size_partials(net, ctx->geo, nullptr))) return rc;
    }
    ctx->cnn = net;
    return IBM_OK;
} IBM_CATCH_ALL

}  // extern "C"
