// Stencil build (Sec. 2.3.1-2.3.2): dead-end filter, compact cut list with the
// axis-projected ghost coefficients of eq. (q_axis), cell classes of
// eq. (dummy_cell_region), and the connected components of the pressure problem
// over open faces (for the compatibility condition and the pressure gauge on
// components that touch no outlet).

#include <hipcub/hipcub.hpp>

#include "common.h"

namespace ibm {
namespace {

struct PopcountOp {
    __host__ __device__ uint32_t operator()(uint8_t m) const { return (uint32_t)__builtin_popcount((unsigned)m); }
};

__global__ void k_set_int(int* p, int v) {
    if (blockIdx.x == 0 && threadIdx.x == 0) *p = v;
}

__global__ void k_zero_bytes(uint8_t* p, long long n) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        p[i] = 0;
}

__device__ inline bool is_dead(const uint16_t* flags, long long c) { return (flags[c] >> 14) & 1; }

// Dead-end filter of eq. (deadend_filter), first pass: a cell whose unfiltered bits
// block five or more of its six directions is a dead end.
__global__ void k_dead_flags(Geo g, const uint8_t* raw, uint16_t* flags, int deadend) {
    long long t0, t1;
    tile_range(g, t0, t1);
    for (long long t = t0; t < t1; ++t) {
        int i, j, k;
        if (!tile_cell(g, t, i, j, k)) continue;
        long long c = cidx(g, i, j, k);
        bool dead = deadend && __builtin_popcount((unsigned)raw[c]) >= 5;
        flags[c] = dead ? (uint16_t)(1u << 14) : (uint16_t)0;
    }
}

// Second pass: a dead-end cell is closed on every non-domain face, and each neighbour
// that saw it through an open face now sees a wall there.
__global__ void k_eff_mask(Geo g, const uint8_t* raw, const uint16_t* flags, uint8_t* eff) {
    long long t0, t1;
    tile_range(g, t0, t1);
    for (long long t = t0; t < t1; ++t) {
        int i, j, k;
        if (!tile_cell(g, t, i, j, k)) continue;
        long long c = cidx(g, i, j, k);
        uint8_t m = raw[c];
        bool dc = is_dead(flags, c);
        for (int d = 0; d < 6; ++d) {
            bool bnd;
            long long nb = nb_index(g, i, j, k, d, bnd);
            if (bnd) continue;
            if (dc || is_dead(flags, nb)) m |= (uint8_t)(1u << d);
        }
        eff[c] = m;
    }
}

// theta seen after the filter: unfiltered cuts keep their theta; a dead cell's new
// cuts have theta 0; a neighbour's new cut toward a dead cell has theta 1 (the dead
// cell's centre); when both cells are dead the smaller value, 0, wins.
__device__ inline double theta_eff(const uint8_t* raw, const uint16_t* flags, const ThetaSrc& theta, long long c,
                                   int d, long long nb) {
    if ((raw[c] >> d) & 1) return theta_of(theta, c, d);
    if (is_dead(flags, c)) return 0.0;
    (void)nb;
    return 1.0;
}

struct CutOut {
    int32_t* cell;
    uint8_t* dir;
    double* theta;
    double* a_ib;
    double* a_c;
    double* a_o;
    int32_t* opp;
};

// One entry per blocked (cell, dir), at cut_off[c] + rank of d among the cell's bits.
// eq. (q_axis): theta >= 0.5 -> q_GC = q_IB/theta + (theta - 1)/theta q_c (theta = 1
// included, q_GC = q_IB); theta < 0.5 -> q_GC = 2 q_IB - 2 theta q_c + (2 theta - 1) q_o
// with q_o the neighbour opposite the cut.  When that opposite face is itself blocked
// or is a domain face, the image point falls back to the cell centre: q_GC = 2 q_IB - q_c.
__global__ void k_fill_cuts(Geo g, const uint8_t* raw, const uint8_t* eff, const uint16_t* flags,
                            const uint32_t* cut_off, ThetaSrc theta, CutOut o) {
    long long t0, t1;
    tile_range(g, t0, t1);
    for (long long t = t0; t < t1; ++t) {
        int i, j, k;
        if (!tile_cell(g, t, i, j, k)) continue;
        long long c = cidx(g, i, j, k);
        uint8_t m = eff[c];
        if (!m) continue;
        uint32_t base = cut_off[c];
        int r = 0;
        for (int d = 0; d < 6; ++d) {
            if (!((m >> d) & 1)) continue;
            uint32_t id = base + r++;
            bool bnd;
            long long nb = nb_index(g, i, j, k, d, bnd);
            double th = theta_eff(raw, flags, theta, c, d, nb);
            int od = d ^ 1;
            bool obnd;
            long long onb = nb_index(g, i, j, k, od, obnd);
            double aib, ac, ao = 0.0;
            int32_t opp = -1;
            if (th >= 0.5) {
                aib = 1.0 / th;
                ac = (th - 1.0) / th;
            } else if (((m >> od) & 1) || obnd) {
                aib = 2.0;
                ac = -1.0;
            } else {
                aib = 2.0;
                ac = -2.0 * th;
                ao = 2.0 * th - 1.0;
                opp = (int32_t)onb;
            }
            o.cell[id] = (int32_t)c;
            o.dir[id] = (uint8_t)d;
            o.theta[id] = th;
            o.a_ib[id] = aib;
            o.a_c[id] = ac;
            o.a_o[id] = ao;
            o.opp[id] = opp;
        }
    }
}

__global__ void k_ncut(const uint32_t* cut_off, const uint8_t* eff, long long N, unsigned long long* out) {
    if (blockIdx.x == 0 && threadIdx.x == 0)
        out[0] = (unsigned long long)cut_off[N - 1] + (unsigned long long)__builtin_popcount((unsigned)eff[N - 1]);
}

// wall-including class: some blocked direction with theta <= 0.5; near bits theta < 0.5
__global__ void k_class_inc(Geo g, const uint8_t* raw, const uint8_t* eff, ThetaSrc theta, uint16_t* flags) {
    long long t0, t1;
    tile_range(g, t0, t1);
    for (long long t = t0; t < t1; ++t) {
        int i, j, k;
        if (!tile_cell(g, t, i, j, k)) continue;
        long long c = cidx(g, i, j, k);
        uint8_t m = eff[c];
        uint16_t f = flags[c] & (uint16_t)(1u << 14);
        bool inc = false;
        uint16_t near = 0;
        for (int d = 0; d < 6; ++d) {
            if (!((m >> d) & 1)) continue;
            bool bnd;
            long long nb = nb_index(g, i, j, k, d, bnd);
            double th = theta_eff(raw, flags, theta, c, d, nb);
            if (th <= 0.5) inc = true;
            if (th < 0.5) near |= (uint16_t)(1u << d);
        }
        f |= (uint16_t)m | (uint16_t)(near << 8);
        if (inc) f |= (uint16_t)(1u << 6);
        flags[c] = f;
    }
}

// wall-adjacent class: not wall-including, with a wall-including face neighbour
__global__ void k_class_adj(Geo g, uint16_t* flags) {
    long long t0, t1;
    tile_range(g, t0, t1);
    for (long long t = t0; t < t1; ++t) {
        int i, j, k;
        if (!tile_cell(g, t, i, j, k)) continue;
        long long c = cidx(g, i, j, k);
        uint16_t f = flags[c];
        if ((f >> 6) & 3) continue;
        bool adj = false;
        for (int d = 0; d < 6; ++d) {
            bool bnd;
            long long nb = nb_index(g, i, j, k, d, bnd);
            if (bnd) continue;
            if (((flags[nb] >> 6) & 3) == 1) adj = true;
        }
        if (adj) flags[c] = f | (uint16_t)(2u << 6);
    }
}

// pressure operator code: open faces (not blocked, not a non-periodic domain face;
// periodic wraps are open) and the number of outlet faces (Dirichlet p = 0)
__global__ void k_pcode(Geo g, const uint8_t* eff, uint8_t* pcode) {
    long long t0, t1;
    tile_range(g, t0, t1);
    for (long long t = t0; t < t1; ++t) {
        int i, j, k;
        if (!tile_cell(g, t, i, j, k)) continue;
        long long c = cidx(g, i, j, k);
        uint8_t m = eff[c];
        unsigned code = 0, outl = 0;
        for (int d = 0; d < 6; ++d) {
            bool bnd;
            (void)nb_index(g, i, j, k, d, bnd);
            if (bnd) {
                if (g.bc[d] == IBM_BC_OUTFLOW) outl += 1;
            } else if (!((m >> d) & 1)) {
                code |= 1u << d;
            }
        }
        pcode[c] = (uint8_t)(code | (outl << 6));
    }
}

__global__ void k_label_init(Geo g, int32_t* label) {
    long long t0, t1;
    tile_range(g, t0, t1);
    for (long long t = t0; t < t1; ++t) {
        int i, j, k;
        if (!tile_cell(g, t, i, j, k)) continue;
        long long c = cidx(g, i, j, k);
        label[c] = (int32_t)c;
    }
}

// Min-label propagation over open faces with hooking of the old root.
__global__ void k_label_prop(Geo g, const uint8_t* eff, int32_t* label, int* changed) {
    long long t0, t1;
    tile_range(g, t0, t1);
    for (long long t = t0; t < t1; ++t) {
        int i, j, k;
        if (!tile_cell(g, t, i, j, k)) continue;
        long long c = cidx(g, i, j, k);
        uint8_t m = eff[c];
        int32_t own = label[c];
        int32_t l = own;
        for (int d = 0; d < 6; ++d) {
            if ((m >> d) & 1) continue;
            bool bnd;
            long long nb = nb_index(g, i, j, k, d, bnd);
            if (bnd) continue;
            int32_t ln = label[nb];
            l = ln < l ? ln : l;
        }
        if (l < own) {
            atomicMin(&label[c], l);
            atomicMin(&label[own], l);
            *changed = 1;
        }
    }
}

__global__ void k_label_jump(Geo g, int32_t* label) {
    long long t0, t1;
    tile_range(g, t0, t1);
    for (long long t = t0; t < t1; ++t) {
        int i, j, k;
        if (!tile_cell(g, t, i, j, k)) continue;
        long long c = cidx(g, i, j, k);
        int32_t l = label[c];
        int32_t ll = label[l];
        while (ll < l) {
            l = ll;
            ll = label[l];
        }
        atomicMin(&label[c], l);
    }
}

__device__ inline bool has_outlet(const Geo& g, int i, int j, int k) {
    if (g.bc[1] == IBM_BC_OUTFLOW && i == g.nx - 1) return true;
    if (g.bc[3] == IBM_BC_OUTFLOW && j == g.ny - 1) return true;
    if (g.bc[5] == IBM_BC_OUTFLOW && k == g.nz - 1) return true;
    return false;
}

__global__ void k_mark_outlet(Geo g, const int32_t* label, uint8_t* has_out) {
    long long t0, t1;
    tile_range(g, t0, t1);
    for (long long t = t0; t < t1; ++t) {
        int i, j, k;
        if (!tile_cell(g, t, i, j, k)) continue;
        if (has_outlet(g, i, j, k)) has_out[label[cidx(g, i, j, k)]] = 1;
    }
}

// enclosed bit; root flag for the component numbering; enclosed-cell flag
__global__ void k_enclosed(Geo g, const int32_t* label, const uint8_t* has_out, uint16_t* flags, int* is_root,
                           int* is_enc) {
    long long t0, t1;
    tile_range(g, t0, t1);
    for (long long t = t0; t < t1; ++t) {
        int i, j, k;
        if (!tile_cell(g, t, i, j, k)) continue;
        long long c = cidx(g, i, j, k);
        int32_t l = label[c];
        bool enc = has_out[l] == 0;
        if (enc) flags[c] |= (uint16_t)(1u << 15);
        is_enc[c] = enc ? 1 : 0;
        is_root[c] = (enc && l == (int32_t)c) ? 1 : 0;
    }
}

__global__ void k_compact(long long N, const int* flag, const int* pos, const int32_t* label, const int* root_id,
                          int32_t* cells, int32_t* keys) {
    for (long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x; c < N; c += (long long)gridDim.x * blockDim.x) {
        if (!flag[c]) continue;
        int p = pos[c];
        cells[p] = (int32_t)c;
        keys[p] = root_id[label[c]];
    }
}

__global__ void k_comp_start(long long n, const int32_t* keys, long long* start, int ncomp) {
    for (long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += (long long)gridDim.x * blockDim.x) {
        if (p == 0 || keys[p] != keys[p - 1]) start[keys[p]] = p;
        if (p == n - 1) start[ncomp] = n;
    }
}

template <class T>
int scan_exclusive(const T* in, T* out, long long n, hipStream_t s) {
    void* tmp = nullptr;
    size_t bytes = 0;
    IBM_HIP(hipcub::DeviceScan::ExclusiveSum(nullptr, bytes, in, out, (int)n, s));
    IBM_HIP(ibm::dev_malloc_async(&tmp, bytes, s));
    IBM_HIP(hipcub::DeviceScan::ExclusiveSum(tmp, bytes, in, out, (int)n, s));
    IBM_HIP(hipFreeAsync(tmp, s));
    return IBM_OK;
}

// a cell with a blocked face (effective mask) or on a non-periodic domain face
struct SpecialCell {
    const uint8_t* mask;
    int nx, ny, nz;
    bool x0, x1, y0, y1, z0, z1;   // the domain face is not periodic
    __host__ __device__ int operator()(int c) const {
        if (mask[c]) return 1;
        const int i = c % nx, r = c / nx, j = r % ny, k = r / ny;
        return ((x0 && i == 0) || (x1 && i == nx - 1) || (y0 && j == 0) || (y1 && j == ny - 1) || (z0 && k == 0) ||
                (z1 && k == nz - 1))
                   ? 1
                   : 0;
    }
};

struct IsSpecial {
    SpecialCell f;
    __host__ __device__ bool operator()(int c) const { return f(c) != 0; }
};

int grow(void** p, size_t bytes) {
    if (*p) IBM_HIP(hipFree(*p));
    *p = nullptr;
    hipError_t e = ibm::dev_malloc(p, bytes < 256 ? 256 : bytes);
    if (e != hipSuccess) {
        set_error("device allocation failed in ibm_build_stencils");
        return IBM_ERR_OOM;
    }
    return IBM_OK;
}

}  // namespace

int stencil_run(ibm_ctx* c, const uint8_t* blocked, const ThetaSrc& theta, int deadend, hipStream_t s) {
    const Geo& g = c->geo;
    const long long N = c->N;
    const int nb = grid_blocks(g);
    int rc;
    k_dead_flags<<<nb, NT, 0, s>>>(g, blocked, c->flags, deadend);
    k_eff_mask<<<nb, NT, 0, s>>>(g, blocked, c->flags, c->mask);
    IBM_HIP(hipGetLastError());
    c->has_dead = deadend ? 1 : 0;

    // cut offsets: exclusive scan of popcount(mask)
    {
        void* tmp = nullptr;
        size_t bytes = 0;
        hipcub::TransformInputIterator<uint32_t, PopcountOp, const uint8_t*> it(c->mask, PopcountOp());
        IBM_HIP(hipcub::DeviceScan::ExclusiveSum(nullptr, bytes, it, c->cut_off, (int)N, s));
        IBM_HIP(ibm::dev_malloc_async(&tmp, bytes, s));
        IBM_HIP(hipcub::DeviceScan::ExclusiveSum(tmp, bytes, it, c->cut_off, (int)N, s));
        IBM_HIP(hipFreeAsync(tmp, s));
    }
    unsigned long long* dncut = (unsigned long long*)c->red;
    k_ncut<<<1, 1, 0, s>>>(c->cut_off, c->mask, N, dncut);
    unsigned long long ncut = 0;
    IBM_HIP(hipMemcpyAsync(&ncut, dncut, sizeof(ncut), hipMemcpyDeviceToHost, s));
    IBM_HIP(hipStreamSynchronize(s));
    if (ncut >= 0xFFFFFFFFull) {
        set_error("ibm_build_stencils: more than 2^32-1 cuts");
        return IBM_ERR_ARG;
    }
    c->ncut = (long long)ncut;
    if ((long long)ncut > c->ncut_cap) {
        long long cap = (long long)ncut + ncut / 8 + 64;
        if ((rc = grow((void**)&c->cut_cell, sizeof(int32_t) * cap))) return rc;
        if ((rc = grow((void**)&c->cut_dir, sizeof(uint8_t) * cap))) return rc;
        if ((rc = grow((void**)&c->cut_theta, sizeof(double) * cap))) return rc;
        if ((rc = grow((void**)&c->a_ib, sizeof(double) * cap))) return rc;
        if ((rc = grow((void**)&c->a_c, sizeof(double) * cap))) return rc;
        if ((rc = grow((void**)&c->a_o, sizeof(double) * cap))) return rc;
        if ((rc = grow((void**)&c->cut_opp, sizeof(int32_t) * cap))) return rc;
        c->ncut_cap = cap;
    }
    CutOut o{c->cut_cell, c->cut_dir, c->cut_theta, c->a_ib, c->a_c, c->a_o, c->cut_opp};
    k_fill_cuts<<<nb, NT, 0, s>>>(g, blocked, c->mask, c->flags, c->cut_off, theta, o);
    k_class_inc<<<nb, NT, 0, s>>>(g, blocked, c->mask, theta, c->flags);
    k_class_adj<<<nb, NT, 0, s>>>(g, c->flags);
    k_pcode<<<nb, NT, 0, s>>>(g, c->mask, c->pcode);
    IBM_HIP(hipGetLastError());

    // connected components over open faces
    int* changed = (int*)c->counter + 8;   // spare slot of the ticket array
    int hchanged = 1;
    k_label_init<<<nb, NT, 0, s>>>(g, c->label);
    int rounds = 0;
    while (hchanged) {
        k_set_int<<<1, 1, 0, s>>>(changed, 0);
        k_label_prop<<<nb, NT, 0, s>>>(g, c->mask, c->label, changed);
        k_label_jump<<<nb, NT, 0, s>>>(g, c->label);
        k_label_jump<<<nb, NT, 0, s>>>(g, c->label);
        IBM_HIP(hipGetLastError());
        IBM_HIP(hipMemcpyAsync(&hchanged, changed, sizeof(int), hipMemcpyDeviceToHost, s));
        IBM_HIP(hipStreamSynchronize(s));
        if (++rounds > 100000) {
            set_error("ibm_build_stencils: component labelling did not converge");
            return IBM_ERR_HIP;
        }
    }

    // enclosed components: no cell with an outlet face
    uint8_t* has_out = (uint8_t*)c->q;            // N bytes of scratch
    int* is_root = (int*)c->r;                    // N ints
    int* is_enc = (int*)c->r + N;                 // N ints (r holds 8N bytes)
    int* root_pos = (int*)c->d;
    int* enc_pos = (int*)c->d + N;
    k_zero_bytes<<<2048, 256, 0, s>>>(has_out, N);
    k_mark_outlet<<<nb, NT, 0, s>>>(g, c->label, has_out);
    k_enclosed<<<nb, NT, 0, s>>>(g, c->label, has_out, c->flags, is_root, is_enc);
    IBM_HIP(hipGetLastError());
    if ((rc = scan_exclusive<int>(is_root, root_pos, N, s))) return rc;
    if ((rc = scan_exclusive<int>(is_enc, enc_pos, N, s))) return rc;
    int last[4];
    IBM_HIP(hipMemcpyAsync(&last[0], root_pos + N - 1, sizeof(int), hipMemcpyDeviceToHost, s));
    IBM_HIP(hipMemcpyAsync(&last[1], is_root + N - 1, sizeof(int), hipMemcpyDeviceToHost, s));
    IBM_HIP(hipMemcpyAsync(&last[2], enc_pos + N - 1, sizeof(int), hipMemcpyDeviceToHost, s));
    IBM_HIP(hipMemcpyAsync(&last[3], is_enc + N - 1, sizeof(int), hipMemcpyDeviceToHost, s));
    IBM_HIP(hipStreamSynchronize(s));
    int ncomp = last[0] + last[1];
    long long nenc = (long long)last[2] + last[3];
    c->ncomp = ncomp;
    c->nenc = nenc;
    if (nenc > 0) {
        if (nenc > c->enc_cap) {
            if ((rc = grow((void**)&c->enc_cells, sizeof(int32_t) * nenc))) return rc;
            c->enc_cap = nenc;
        }
        if (ncomp + 1 > c->comp_cap) {
            if ((rc = grow((void**)&c->comp_start, sizeof(long long) * (ncomp + 1)))) return rc;
            c->comp_cap = ncomp + 1;
        }
        int32_t *cells_in = nullptr, *keys_in = nullptr, *keys_out = nullptr;
        IBM_HIP(ibm::dev_malloc_async((void**)&cells_in, sizeof(int32_t) * nenc, s));
        IBM_HIP(ibm::dev_malloc_async((void**)&keys_in, sizeof(int32_t) * nenc, s));
        IBM_HIP(ibm::dev_malloc_async((void**)&keys_out, sizeof(int32_t) * nenc, s));
        k_compact<<<4096, 256, 0, s>>>(N, is_enc, enc_pos, c->label, root_pos, cells_in, keys_in);
        IBM_HIP(hipGetLastError());
        void* tmp = nullptr;
        size_t bytes = 0;
        int endbit = 1;
        while ((1ll << endbit) < (long long)ncomp + 1 && endbit < 32) ++endbit;
        IBM_HIP(hipcub::DeviceRadixSort::SortPairs(nullptr, bytes, keys_in, keys_out, cells_in, c->enc_cells,
                                                   (int)nenc, 0, endbit, s));
        IBM_HIP(ibm::dev_malloc_async(&tmp, bytes, s));
        IBM_HIP(hipcub::DeviceRadixSort::SortPairs(tmp, bytes, keys_in, keys_out, cells_in, c->enc_cells,
                                                   (int)nenc, 0, endbit, s));
        k_comp_start<<<4096, 256, 0, s>>>(nenc, keys_out, c->comp_start, ncomp);
        IBM_HIP(hipGetLastError());
        IBM_HIP(hipFreeAsync(tmp, s));
        IBM_HIP(hipFreeAsync(cells_in, s));
        IBM_HIP(hipFreeAsync(keys_in, s));
        IBM_HIP(hipFreeAsync(keys_out, s));
    }
    // the special-cell list of the step kernels (count, size, select in cell order)
    {
        c->spec_ready = false;
        const SpecialCell f{c->mask, g.nx, g.ny, g.nz, g.bc[0] != IBM_BC_PERIODIC, g.bc[1] != IBM_BC_PERIODIC,
                            g.bc[2] != IBM_BC_PERIODIC, g.bc[3] != IBM_BC_PERIODIC, g.bc[4] != IBM_BC_PERIODIC,
                            g.bc[5] != IBM_BC_PERIODIC};
        hipcub::CountingInputIterator<int> cells(0);
        hipcub::TransformInputIterator<int, SpecialCell, hipcub::CountingInputIterator<int>> flags(cells, f);
        int* dcount = (int*)c->counter + 10;   // spare slot of the ticket array
        void* tmp = nullptr;
        size_t bytes = 0;
        IBM_HIP(hipcub::DeviceReduce::Sum(nullptr, bytes, flags, dcount, (int)N, s));
        IBM_HIP(ibm::dev_malloc_async(&tmp, bytes, s));
        IBM_HIP(hipcub::DeviceReduce::Sum(tmp, bytes, flags, dcount, (int)N, s));
        IBM_HIP(hipFreeAsync(tmp, s));
        int hcount = 0;
        IBM_HIP(hipMemcpyAsync(&hcount, dcount, sizeof(int), hipMemcpyDeviceToHost, s));
        IBM_HIP(hipStreamSynchronize(s));
        c->nspec = hcount;
        if (hcount > c->spec_cap) {
            if ((rc = grow((void**)&c->spec_cells, sizeof(int32_t) * (size_t)hcount))) return rc;
            c->spec_cap = hcount;
        }
        if (hcount > 0) {
            tmp = nullptr;
            bytes = 0;
            IBM_HIP(hipcub::DeviceSelect::If(nullptr, bytes, cells, c->spec_cells, dcount, (int)N, IsSpecial{f}, s));
            IBM_HIP(ibm::dev_malloc_async(&tmp, bytes, s));
            IBM_HIP(hipcub::DeviceSelect::If(tmp, bytes, cells, c->spec_cells, dcount, (int)N, IsSpecial{f}, s));
            IBM_HIP(hipFreeAsync(tmp, s));
        }
        c->spec_ready = true;
    }
    c->stencil_ready = true;
    return IBM_OK;
}

}  // namespace ibm
