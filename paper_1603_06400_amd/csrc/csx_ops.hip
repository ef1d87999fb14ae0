// csx_ops.hip -- forward and adjoint operators of the fan-beam coded-aperture
// coherent-scatter model on gfx950 (Odinaka et al., arXiv:1603.06400).
//
//   g_i  = sum_j A_ij T_ij sum_m q_m Phi(kappa_ij q_m) f_jm          (forward, Alg. 1)
//   b_jm = q_m sum_i A_ij T_ij Phi(kappa_ij q_m) y_i                 (adjoint, Alg. 3)
//   kappa = hc / sin(theta/2)   (E = kappa q, Bragg's law, App. A)
//   A = C Gso God dtheta (1 + cos^2 theta) cos(theta/2) / sin^2(theta/2)
//
// Work decomposition (wave64):
//  * a "class" is a set of pairs that share every factor except the mask
//    transmission T: the pixel rows y' and -y' (up-down mirror, Sec. III-A)
//    and, when the voxel grid and the detector are centred with even sizes,
//    the voxel / pixel columns x and -x (left-right mirror).  One class is
//    4 pairs (2 without the left-right mirror); its four mask cells come from a
//    single crossing point, mirrored with integer arithmetic.
//  * lane = class.  Each lane evaluates its class's factors once and keeps
//    kappa and the pair weights in its own registers; the q loop then runs
//    inside the lane (fully unrolled over a chunk of <= 64 q), so no lane ever
//    waits on a value another lane produced.  On a uniform q grid the per-q
//    step is one FP64 add for the Bragg bin coordinate (an FMA anchors it at
//    the first node of each 16-node block), its conversion to an integer, a
//    gather from the spectrum table in LDS and FP32 FMAs; the table carries
//    zero pads wide enough for every coordinate a wave can reach (sized on
//    the host from the band test), so no clamp is needed.  On a non-uniform
//    grid q/dE comes from scalar loads and each index is clamped onto the
//    table's two zero pads.
//  * q blocks (16 nodes on a uniform grid, 8 otherwise) are skipped, uniformly
//    for the wave, when no lane's Bragg energies kappa q can reach the
//    spectrum band there (one ballot per block).
//  * the spectral bin of a triple is decided in float64 (kappa in float64
//    from float32 seeds refined by one Newton step each; the bin coordinate
//    q/dE * kappa + 1 - e_lo/dE by FP64 FMA, or on a uniform grid by an FMA
//    at each block's first node and FP64 adds between): float64 precision,
//    so bin decisions agree with the float64 definition except within
//    ~1e-13 of a bin edge.
//  * adjoint: one wave per voxel (and its x-mirror) walks the pixel classes 64
//    at a time, accumulating per-lane partial images acc[q]; one butterfly
//    transpose-reduction per wave sums them over lanes (no atomics).
//  * forward: one wave per group of mirror pixels; one lane per voxel (pair)
//    evaluates both mirror classes and accumulates the paper's W(r, theta) =
//    sum_q S f over the q chunk, reading q f from a q-major LDS tile shared by
//    the block (double-buffered, the next tile's loads in flight during the
//    current one); the voxel range is split across blocks, numbered so that
//    each XCD reads its own share of f, and the partial images are summed in
//    a fixed order (bitwise reproducible).
#include "csx_internal.h"

#include "csx_device.h"

// q nodes per skip block of the uniform-grid loops (adjoint, forward),
// capped at the chunk width
constexpr int QB_ADJ = 16;
constexpr int QB_FWD = 16;
// q nodes per skip block when the factor store supplies each tile's node
// range (a wave-uniform scalar test per block, no ballot)
constexpr int QB_ST = 4;

namespace {

// ---------------------------------------------------------------------------
// adjoint: one wave per voxel group (voxel j, and its mirror j2 with LR) and
// q chunk; lanes = pixel classes (a, b_up), b_up in the upper half, 64 per batch.
// ---------------------------------------------------------------------------
// EN = 1: energy-resolved data (the energy-sensitive detector of App. A).
// rho is then Psi [ne + 2][npix], Psi[k][i] = Phi_k y_E[k - 1][i] with zero
// planes at the pad bins 0 and ne + 1, and a triple reads Psi at its own
// spectrum bin and pixel instead of Phi times the pixel's ratio.
// ST = 1: the class factors come from the factor store (T.ra) instead of
// being evaluated: the same values, computed once per geometry by
// k_store_adjoint with the same code.
template <int LR, int QW, int QU, int EN = 0, int ST = 0>
__device__ __forceinline__ void adjoint_body(const KParams &P, const DevTables &T, const Lds &L,
                                             const double *__restrict__ qa,
                                             const double2 *__restrict__ qblk,
                                             const float *__restrict__ rho, float *__restrict__ b,
                                             int bx, int by, int bz = 0)
{
    static_assert(!(EN && ST), "the energy-resolved adjoint evaluates its factors");
    constexpr int NB = QW / 8;
    extern __shared__ __align__(16) unsigned char lds[];
    float *s_phi = (float *)(lds + L.phi) + P.spec_lo;   // entry 0 of the padded table
    uint32_t *s_bits = (uint32_t *)(lds + L.mask);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;

    stage_tables(P, T, (float *)(lds + L.phi), s_bits);
    // wave-uniform (readfirstlane): the voxel records load into scalar
    // registers.  The wave's first global reads (voxel records, the first
    // tile's detector values and records, the output node) are issued before
    // the tables' barrier; a wave past the last group reads group 0's and
    // leaves after it.
    const int g_w = __builtin_amdgcn_readfirstlane(bx * (blockDim.x >> 6) + wv);
    const bool live = g_w < P.n_groups;
    const int g = live ? g_w : 0;

    int j, j2;
    if (LR) {
        const int half = P.nx / 2;
        const int iz = g / half, ix = g % half;
        j = iz * P.nx + ix;
        j2 = iz * P.nx + (P.nx - 1 - ix);
    } else {
        j = g;
        j2 = g;
    }
    const VoxD vd = T.vd[j];
    const float2 vf = T.vf[j];
    const double2 vm = T.vm[j];
    const int m0 = by * QW;
    const double *qa_c = qa + m0;
    const double2 *qb_c = qblk + by * NB;
    const double b0 = P.b0;
    const uint32_t top = (uint32_t)(P.ne + 1);

    float acc0[QW], acc1[QW];
#pragma unroll
    for (int m = 0; m < QW; ++m) {
        acc0[m] = 0.0f;
        acc1[m] = 0.0f;
    }

    // pixel classes in 8 x 8 tiles (columns a, upper rows bu): neighbouring
    // pixels have close scatter angles, so the q-block skip is tighter
    const int half_y = P.ndy / 2;
    const int ntx = (P.ndx + 7) / 8;
    const int ntiles = P.cls_list ? (P.n_cls + 63) / 64 : ntx * ((half_y + 7) / 8);
    const int lx = lane & 7, ly = lane >> 3;
    // class (column a, upper row r) of the lane in tile t: an 8 x 8 tile of
    // the detector, or 64 consecutive entries of the class list
    auto class_of = [&](int t, int &a, int &r) -> bool {
        if (P.cls_list) {
            const int e = t * 64 + lane;
            if (e >= P.n_cls) return false;
            const int c = P.cls_list[e];
            a = c % P.ndx;
            r = c / P.ndx;
            return true;
        }
        a = (t % ntx) * 8 + lx;
        r = (t / ntx) * 8 + ly;
        return a < P.ndx && r < half_y;
    };
    // detector values of the lane's class (and with ST its stored record),
    // prefetched one tile ahead
    float r_u = 0.0f, r_d = 0.0f, r_bu = 0.0f, r_bd = 0.0f;
    const int ntiles_all = ntx * ((half_y + 7) / 8);
    double rk = 0.0;
    float rA = 0.0f;
    uint32_t rb = 0u, rtm = 0u;
    auto load_rho = [&](int t) {
        int a, r;
        if (EN) return;                         // read per node from Psi
        if (ST) {
            rb = 0u;
            // the tile's node range: a superset of its lanes' ranges, from
            // the store's tile record (wave-uniform)
            if (QU && (P.ra_gs || !P.cls_list))
                rtm = __builtin_amdgcn_readfirstlane(
                    T.ram[P.ra_gs ? ((size_t)g * P.ra_gs + (size_t)t * 64) / 64 : (size_t)g * ntiles_all + t]);
        }
        if (class_of(t, a, r)) {
            if (ST) {
                // record of class (a, r): tile (r/8, a/8), lane 8 (r mod 8) + a mod 8,
                // or entry t 64 + lane of a list-order store
                const size_t e = P.ra_gs ? (size_t)g * P.ra_gs + (size_t)t * 64 + lane
                                         : ((size_t)g * ntiles_all + (r >> 3) * ntx + (a >> 3)) * 64 +
                                               ((r & 7) << 3) + (a & 7);
                const uint4 v = load_nt(T.ra + e);
                rk = __longlong_as_double((long long)(((uint64_t)v.y << 32) | v.x));
                rA = __uint_as_float(v.z);
                rb = v.w;
            }
            const int bu = half_y + r;
            const int bd = P.ndy - 1 - bu;
            r_u = rho[bu * P.ndx + a];
            r_d = rho[bd * P.ndx + a];
            if (LR) {
                const int ab = P.ndx - 1 - a;
                r_bu = rho[bu * P.ndx + ab];
                r_bd = rho[bd * P.ndx + ab];
            }
        }
    };
    // split adjoint: this wave's contiguous range of tiles, into partial image bz
    int tb = 0, te = ntiles;
    if (P.asplit > 1 && !P.cls_list) {
        const int per = (ntiles + P.asplit - 1) / P.asplit;
        tb = min(ntiles, bz * per);
        te = min(ntiles, tb + per);
        b += (size_t)bz * P.nvox * P.nq;
    }
    if (tb < te) load_rho(tb);
    // the lane's output node after the q reduction, and its q value
    const int m_out = m0 + transposed_index<QW>(lane);
    const bool writer = (lane & ((64 / QW) - 1)) == 0 && m_out < P.nq;
    const float qm = writer ? T.qv[m_out] : 0.0f;
    __syncthreads();
    if (!live) return;

    for (int t = tb; t < te; ++t) {
        const uint32_t tm_cur = rtm;   // the tile's node range (store), read ahead with its records
        (void)tm_cur;
        int a = 0, r = 0;
        const bool has = class_of(t, a, r);
        double kap = 0.0;
        float c0 = 0.0f, c1 = 0.0f;
        bool act = false;
        // EN: the class's pair weight times each pixel's mask value, and the
        // pixels' columns in Psi
        float eu = 0.0f, ed = 0.0f, ebu = 0.0f, ebd = 0.0f;
        const float *pu = rho, *pd = rho, *pbu = rho, *pbd = rho;
        if (ST) {
            // as below, with A, kappa and the mask values read from the store
            if (has && (rb & CSX_REC_ACT)) {
                const float tu = (float)(rb & 1u), td = (float)((rb >> 1) & 1u);
                const float w0 = tu * r_u + td * r_d;
                float w1 = 0.0f;
                if (LR) {
                    const float tbu = (float)((rb >> 2) & 1u), tbd = (float)((rb >> 3) & 1u);
                    w1 = tbu * r_bu + tbd * r_bd;
                }
                if (w0 != 0.0f || w1 != 0.0f) {
                    c0 = rA * w0;
                    c1 = rA * w1;
                    act = c0 != 0.0f || c1 != 0.0f;
                    if (act) kap = rk;
                }
            }
        } else if (has) {
            const int bu = half_y + r;
            const double xp = pixel_coord(P, a, P.ndx);
            const double yp = pixel_coord(P, bu, P.ndy);
            const Cells c = mask_cells(P, vm, xp, yp);
            float w0 = 0.0f, w1 = 0.0f;
            float tu = 0.0f, td = 0.0f, tbu = 0.0f, tbd = 0.0f;
            if (c.in_rows) {
                const uint32_t ru = s_bits[c.row_u], rd = s_bits[c.row_d];
                tu = bitf(ru, c.col_a);
                td = bitf(rd, c.col_a);
                if (LR) {
                    tbu = bitf(ru, c.col_b);
                    tbd = bitf(rd, c.col_b);
                }
                if (EN) {
                    w0 = tu + td;
                    w1 = tbu + tbd;
                } else {
                    w0 = tu * r_u + td * r_d;
                    if (LR) w1 = tbu * r_bu + tbd * r_bd;
                }
            }
            if (w0 != 0.0f || w1 != 0.0f) {
                double k;
                float A;
                pair_factors(P, vd, vf, xp, yp, k, A);
                if (in_band(P, k)) {
                    c0 = A * w0;
                    c1 = A * w1;
                    act = c0 != 0.0f || c1 != 0.0f;
                    if (act) kap = k;
                    if (EN) {
                        const int bd = P.ndy - 1 - bu;
                        eu = A * tu;
                        ed = A * td;
                        pu = rho + bu * P.ndx + a;
                        pd = rho + bd * P.ndx + a;
                        if (LR) {
                            const int ab = P.ndx - 1 - a;
                            ebu = A * tbu;
                            ebd = A * tbd;
                            pbu = rho + bu * P.ndx + ab;
                            pbd = rho + bd * P.ndx + ab;
                        }
                    }
                }
            }
        }
        // EN: sum over the class's pixels of A T Psi[kk][pixel] (zero weights
        // skip their loads)
        auto psi_sum = [&](uint32_t kk, float e1, const float *p1, float e2, const float *p2) -> float {
            const size_t o = (size_t)kk * P.npix;
            float v = 0.0f;
            if (e1 != 0.0f) v = e1 * p1[o];
            if (e2 != 0.0f) v = fmaf(e2, p2[o], v);
            return v;
        };
        // the class's values at its current bin, reloaded only when the bin
        // changes (consecutive q nodes share a bin); pad bins are 0
        uint32_t cur = 0u;
        float v0 = 0.0f, v1 = 0.0f;
        auto en_node = [&](uint32_t kk) {
            if (kk != cur) {
                cur = kk;
                const bool pad = kk == 0u || kk == top;
                v0 = pad ? 0.0f : psi_sum(kk, eu, pu, ed, pd);
                if (LR) v1 = pad ? 0.0f : psi_sum(kk, ebu, pbu, ebd, pbd);
            }
        };
        if (t + 1 < te) load_rho(t + 1);
        if (__ballot(act) == 0) continue;
        if (QU) {
            // uniform q grid: u_m = u0 + m du, in-band nodes in the wave's range
            const double u0 = fma(kap, P.a0 + P.da * m0, b0), du = kap * P.da;
            int lo = QW, hi = -1;
            if (ST) {
                // the tile's node range (a superset of its lanes' ranges),
                // wave-uniform: from the store's tile record, or reduced over
                // the lanes for a class list
                if (P.cls_list && !P.ra_gs) {
                    if (act) band_range(P, u0, du, 0, QW, lo, hi);
                    lo = wave_min(lo);
                    hi = wave_max(hi);
                } else {
                    lo = (int)(tm_cur & 0xffffu) - m0;
                    hi = (int)(tm_cur >> 16) - m0;
                }
            } else if (act) {
                band_range(P, u0, du, 0, QW, lo, hi);
            }
            constexpr int BA = ST ? QB_ST : (QB_ADJ < QW ? QB_ADJ : QW);
#pragma unroll
            for (int blk = 0; blk < QW / BA; ++blk) {
                // skip a block no lane of the wave has in band (its triples add exact zeros)
                if (ST) {
                    if (blk * BA + BA - 1 < lo || blk * BA > hi) continue;
                } else if (__ballot(lo <= blk * BA + BA - 1 && hi >= blk * BA) == 0) {
                    continue;
                }
                // anchored by an FMA at each block's first node, then one add per node
                double u = fma((double)(blk * BA), du, u0);
#pragma unroll
                for (int mm = 0; mm < BA; ++mm) {
                    const int m = blk * BA + mm;
                    // the table's pads cover every coordinate: no clamp unless
                    // the bin indexes the energy data
                    const int ku = (int)u;
                    const uint32_t kk = min((uint32_t)ku, top);
                    u += du;
                    if (EN) {
                        en_node(kk);
                        acc0[m] += v0;
                        if (LR) acc1[m] += v1;
                    } else {
                        const float ph = s_phi[ku];
                        acc0[m] = fmaf(c0, ph, acc0[m]);
                        if (LR) acc1[m] = fmaf(c1, ph, acc1[m]);
                    }
                }
            }
        } else {
#pragma unroll
            for (int blk = 0; blk < NB; ++blk) {
                const double2 qr = qb_c[blk];
                const bool need = act && kap * qr.y >= P.band_lo && kap * qr.x < P.band_hi;
                if (__ballot(need) == 0) continue;
#pragma unroll
                for (int mm = 0; mm < 8; ++mm) {
                    const int m = blk * 8 + mm;
                    const uint32_t kk = spec_index(kap, qa_c[m], b0, top);
                    if (EN) {
                        en_node(kk);
                        acc0[m] += v0;
                        if (LR) acc1[m] += v1;
                    } else {
                        const float ph = spec(s_phi, kk);
                        acc0[m] = fmaf(c0, ph, acc0[m]);
                        if (LR) acc1[m] = fmaf(c1, ph, acc1[m]);
                    }
                }
            }
        }
    }
    WaveTransposeSum<QW, 32>::run(acc0, lane);
    if (LR) WaveTransposeSum<QW, 32>::run(acc1, lane);
    (void)qb_c;
    if (writer) {
        b[(size_t)j * P.nq + m_out] = acc0[0] * qm;
        if (LR) b[(size_t)j2 * P.nq + m_out] = acc1[0] * qm;
    }
}

// ---------------------------------------------------------------------------
// forward: one wave per output group (the four mirror pixels (+-x', +-y') with
// LR, else the two pixels (x', +-y')) and q chunk; lane = voxel group (64 per
// batch) evaluating both mirror classes; the block's 8 waves share a q-major
// tile of q f for the batch's voxels; blockIdx.y splits the voxel groups.
// ---------------------------------------------------------------------------
// EN = 1: energy-resolved output (the energy-sensitive detector of App. A).
// Each lane adds a triple's contribution to the spectrum bin of its Bragg
// energy instead of summing over bins: consecutive q nodes of a class that
// fall in one bin form a run, and each run is added once per output pixel
// into the wave's histograms in LDS (4 pixels x (ne + 2) bins, 64-bit fixed
// point with the launch's scale sc[0] = 2^s, sc[1] = 2^-s: integer atomics,
// totals independent of the add order).  part then holds [ne][npix] per
// partial image.
// ST = 1: the two classes' factors come from the factor store (T.rf),
// computed once per geometry by k_store_forward with the same code.
template <int LR, int QW, int QU, int EN = 0, int ST = 0>
__device__ __forceinline__ void forward_body(const KParams &P, const DevTables &T, const Lds &L,
                                             const double *__restrict__ qa,
                                             const double2 *__restrict__ qblk,
                                             const float *__restrict__ f,
                                             float *__restrict__ part, int tiles_per_split,
                                             int bx, int by, int bz, int gz,
                                             const double *__restrict__ sc = nullptr)
{
    static_assert(!(EN && ST), "the energy-resolved forward evaluates its factors");
    constexpr int NB = QW / 8;
    constexpr int RPG = LR ? 2 : 1;             // voxel rows per group
    constexpr int ROWS = 64 * RPG;              // tile rows per batch
    constexpr int TS = ROWS + 2;                // tile stride per q (floats), keeps 8-byte alignment
    constexpr int RSTEP = 512 / QW;             // rows staged per pass
    constexpr int NPASS = ROWS / RSTEP;
    extern __shared__ __align__(16) unsigned char lds[];
    float *s_phi = (float *)(lds + L.phi) + P.spec_lo;   // entry 0 of the padded table
    uint32_t *s_bits = (uint32_t *)(lds + L.mask);
    float *s_tile = (float *)(lds + L.tile);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;

    stage_tables(P, T, (float *)(lds + L.phi), s_bits);
    const int NE2 = P.ne + 2;
    unsigned long long *hist = EN ? (unsigned long long *)(lds + L.hist) + (size_t)wv * 4 * NE2 : nullptr;
    if (EN)
        for (int k = lane; k < 4 * NE2; k += 64) hist[k] = 0ull;
    const double fx_scale = EN ? sc[0] : 0.0;
    const int fx_exp = EN ? scale_exponent(fx_scale) : 0;
    auto fx = [&](float v) -> unsigned long long { return fixed_of(v, fx_exp); };

    // wave-uniform (readfirstlane): the pixel quad's values live in scalar registers
    const int quad = __builtin_amdgcn_readfirstlane(bx * 8 + wv);   // 8 waves per block
    const bool wave_on = quad < P.n_quad;
    const int qq = wave_on ? (P.quad_list ? P.quad_list[quad] : quad) : 0;
    int a, bu;
    if (LR) {
        const int hx = P.ndx / 2;
        a = hx + qq % hx;
        bu = P.ndy / 2 + qq / hx;
    } else {
        a = qq % P.ndx;
        bu = P.ndy / 2 + qq / P.ndx;
    }
    const double xpa = pixel_coord(P, a, P.ndx);
    const double yp = pixel_coord(P, bu, P.ndy);
    const int qc = bz;
    const int m0 = qc * QW;
    const double *qa_c = qa + m0;
    const double2 *qb_c = qblk + qc * NB;
    const double b0 = P.b0;
    const uint32_t top = (uint32_t)(P.ne + 1);
    // voxel groups in 8 x 8 tiles (ix over the group columns, iz); blockIdx.y
    // takes a contiguous range of tiles
    const int gw = LR ? P.nx / 2 : P.nx;       // group columns
    const int ntx = (gw + 7) / 8;
    const int ntiles = ntx * ((P.nz + 7) / 8);
    const int t0 = by * tiles_per_split;
    const int t1 = min(ntiles, t0 + tiles_per_split);

    // staging of q f: thread t loads q index t % QW of tile rows t / QW + k * RSTEP
    // (coalesced along q) for the next tile while the current one runs; tile
    // row r holds group r / RPG (lane index), voxel j (r even) or its mirror
    const int sm = threadIdx.x % QW;
    const int sr = threadIdx.x / QW;
    const float qs = (m0 + sm < P.nq) ? T.qv[m0 + sm] : 0.0f;
    float pre[NPASS];
    // (raw f values; the q factor is applied when the tile is written to LDS).
    // A tile and q chunk wholly inside the grid (a block-uniform test) loads
    // without per-value checks, so the loads issue together and their latency
    // overlaps the current tile's work.
    // In-grid tiles: row r = sr + k RSTEP of the tile is group gl = sr/RPG +
    // k G (G = RSTEP/RPG), at column offset (gl mod 8) and row offset gl/8;
    // RSTEP is even, so every row of a thread is a mirror row or none is.
    // With sr/RPG < 8 when G = 4 and G a multiple of 8 otherwise, the offsets
    // split as (g0 mod 8) + a_k and g0/8 + b_k, a_k = kG mod 8, b_k = kG/8:
    // one 32-bit byte offset per thread and tile plus a per-k constant.
    constexpr int G = RSTEP / RPG;
    const int g0 = sr / RPG;
    const bool mir = LR && (sr & 1);
    const uint32_t row_bytes = (uint32_t)P.nx * P.nq * 4u;          // one voxel row of f
    const int col_bytes = (mir ? -P.nq : P.nq) * 4;                 // one voxel column, signed
    auto stage_load = [&](int t) {
        const int tx = t % ntx, ty = t / ntx;
        if (tx * 8 + 8 <= gw && ty * 8 + 8 <= P.nz && m0 + QW <= P.nq) {
            const int ix0 = tx * 8 + (g0 & 7);
            const int col = mir ? (P.nx - 1 - ix0) : ix0;
            const uint32_t e0 = (uint32_t)(((ty * 8 + (g0 >> 3)) * P.nx + col) * P.nq + m0 + sm) * 4u;
            const char *fb = (const char *)f;
#pragma unroll
            for (int k = 0; k < NPASS; ++k) {
                const int ak = (k * G) & 7, bk = (k * G) >> 3;
                const uint32_t o = e0 + (uint32_t)bk * row_bytes + (uint32_t)(ak * col_bytes);
                pre[k] = *(const float *)(fb + o);
            }
        } else {
#pragma unroll
            for (int k = 0; k < NPASS; ++k) {
                const int r = sr + k * RSTEP;
                const int gl = r / RPG;
                const int ix = tx * 8 + (gl & 7), iz = ty * 8 + (gl >> 3);
                float v = 0.0f;
                if (ix < gw && iz < P.nz && m0 + sm < P.nq) {
                    const int vox = iz * P.nx + ((LR && (r & 1)) ? (P.nx - 1 - ix) : ix);
                    v = f[(size_t)vox * P.nq + m0 + sm];
                }
                pre[k] = v;
            }
        }
    };
    // voxel records of the lane's group (with ST the stored class records of
    // (quad, group)), prefetched one tile ahead
    VoxD nvd = {0.0, 1.0, 1.0, 0.0};
    float2 nvf = {0.0f, 0.0f};
    double2 nvm = {0.0, 0.0};
    bool nvalid = false;
    uint4 nr0 = make_uint4(0u, 0u, 0u, 0u), nr1 = make_uint4(0u, 0u, 0u, 0u);
    auto load_vox = [&](int t) {
        const int ix = (t % ntx) * 8 + (lane & 7), iz = (t / ntx) * 8 + (lane >> 3);
        nvalid = ix < gw && iz < P.nz;
        if (ST) {
            if (nvalid) {
                const size_t e = (((size_t)qq * ntiles + t) * 64 + lane) * 2;
                nr0 = load_nt(T.rf + e);
                nr1 = load_nt(T.rf + e + 1);
            }
        } else if (nvalid) {
            const int j = iz * P.nx + ix;
            nvd = T.vd[j];
            nvf = T.vf[j];
            nvm = T.vm[j];
        }
    };
    if (t0 < t1) {
        stage_load(t0);
        load_vox(t0);
    }

    // The energy-integrating forward double-buffers the q f tile (the next
    // tile is written into the idle buffer after the current one is used: one
    // block barrier per tile); the energy mode, whose histograms also live in
    // LDS, keeps one buffer and two barriers.
    constexpr bool DB = !EN;
    constexpr int TBUF = QW * TS;
    auto put_tile = [&](float *dst) {
#pragma unroll
        for (int k = 0; k < NPASS; ++k) dst[sm * TS + sr + k * RSTEP] = qs * pre[k];
    };
    float o0 = 0.0f, o1 = 0.0f, o2 = 0.0f, o3 = 0.0f;
    for (int t = t0; t < t1; ++t) {
        float *tile = s_tile + (DB ? ((t - t0) & 1) * TBUF : 0);
        if (!DB) {
            __syncthreads();
            put_tile(tile);
            __syncthreads();
        } else if (t == t0) {
            put_tile(tile);
            __syncthreads();
        }
        const VoxD vd = nvd;
        const float2 vf = nvf;
        const double2 vm = nvm;
        const bool valid = nvalid;
        const uint4 r0 = nr0, r1 = nr1;
        // ST: node range of the (quad, tile) pair, low 16 bits first node, high 16 bits last
        const uint32_t tmeta = ST ? __builtin_amdgcn_readfirstlane(T.rfm[(size_t)qq * ntiles + t]) : 0u;
        if (t + 1 < t1) {
            stage_load(t + 1);
            load_vox(t + 1);
        }
        // the tile's work; a `continue` below leaves this block only, so the
        // staging of the next tile and its barrier are reached by every thread
        do {
        if (!wave_on) continue;

        // the lane's two classes: pixel column a (class 1) and its mirror (class 2)
        double k1 = 0.0, k2 = 0.0;
        float c10 = 0.0f, c11 = 0.0f, c12 = 0.0f, c13 = 0.0f;
        float c20 = 0.0f, c21 = 0.0f, c22 = 0.0f, c23 = 0.0f;
        bool act1 = false, act2 = false;
        if (ST) {
            // as below, with A, kappa and the mask values read from the store
            const uint32_t rb = r1.z;
            if (valid && (rb & CSX_REC_ACT)) {
                const float A = __uint_as_float(r1.x);
                act1 = true;
                k1 = __longlong_as_double((long long)(((uint64_t)r0.y << 32) | r0.x));
                c10 = A * (float)(rb & 1u);
                c11 = A * (float)((rb >> 1) & 1u);
                c12 = A * (float)((rb >> 2) & 1u);
                c13 = A * (float)((rb >> 3) & 1u);
            }
            if (LR && valid && (rb & (CSX_REC_ACT << 8))) {
                const float A = __uint_as_float(r1.y);
                act2 = true;
                k2 = __longlong_as_double((long long)(((uint64_t)r0.w << 32) | r0.z));
                // O0, O1 <- mirror voxel (column a); O2, O3 <- voxel j (column -a)
                c20 = A * (float)((rb >> 10) & 1u);
                c21 = A * (float)((rb >> 11) & 1u);
                c22 = A * (float)((rb >> 8) & 1u);
                c23 = A * (float)((rb >> 9) & 1u);
            }
        } else if (valid) {
            {
                const Cells c = mask_cells(P, vm, xpa, yp);
                float tau = 0.0f, tad = 0.0f, tbu = 0.0f, tbd = 0.0f;
                if (c.in_rows) {
                    const uint32_t ru = s_bits[c.row_u], rd = s_bits[c.row_d];
                    tau = bitf(ru, c.col_a);
                    tad = bitf(rd, c.col_a);
                    if (LR) {
                        tbu = bitf(ru, c.col_b);
                        tbd = bitf(rd, c.col_b);
                    }
                }
                if (tau + tad + tbu + tbd != 0.0f) {
                    double k;
                    float A;
                    pair_factors(P, vd, vf, xpa, yp, k, A);
                    if (in_band(P, k)) {
                        act1 = true;
                        k1 = k;
                        // O0, O1 <- voxel j (column a); O2, O3 <- mirror voxel (column -a)
                        c10 = A * tau; c11 = A * tad; c12 = A * tbu; c13 = A * tbd;
                    }
                }
            }
            if (LR) {
                const Cells c = mask_cells(P, vm, -xpa, yp);
                float tau = 0.0f, tad = 0.0f, tbu = 0.0f, tbd = 0.0f;
                if (c.in_rows) {
                    const uint32_t ru = s_bits[c.row_u], rd = s_bits[c.row_d];
                    tau = bitf(ru, c.col_a);
                    tad = bitf(rd, c.col_a);
                    tbu = bitf(ru, c.col_b);
                    tbd = bitf(rd, c.col_b);
                }
                if (tau + tad + tbu + tbd != 0.0f) {
                    double k;
                    float A;
                    pair_factors(P, vd, vf, -xpa, yp, k, A);
                    if (in_band(P, k)) {
                        act2 = true;
                        k2 = k;
                        // O0, O1 <- mirror voxel (column a); O2, O3 <- voxel j (column -a)
                        c20 = A * tbu; c21 = A * tbd; c22 = A * tau; c23 = A * tad;
                    }
                }
            }
        }
        if (__ballot(act1 || act2) == 0) continue;
        float w1a = 0.0f, w1b = 0.0f, w2a = 0.0f, w2b = 0.0f;
        const float *trow = tile + lane * RPG;
        // EN: the current run of each class (bin 0 is a pad: no run yet)
        uint32_t cur1 = 0u, cur2 = 0u;
        float r1a = 0.0f, r1b = 0.0f, r2a = 0.0f, r2b = 0.0f;
        auto flush1 = [&]() {
            unsigned long long *hb = hist + cur1;
            if (r1a != 0.0f) {
                if (c10 != 0.0f) atomicAdd(hb, fx(c10 * r1a));
                if (c11 != 0.0f) atomicAdd(hb + NE2, fx(c11 * r1a));
            }
            if (LR && r1b != 0.0f) {
                if (c12 != 0.0f) atomicAdd(hb + 2 * NE2, fx(c12 * r1b));
                if (c13 != 0.0f) atomicAdd(hb + 3 * NE2, fx(c13 * r1b));
            }
            r1a = 0.0f;
            r1b = 0.0f;
        };
        auto flush2 = [&]() {
            unsigned long long *hb = hist + cur2;
            if (r2b != 0.0f) {
                if (c20 != 0.0f) atomicAdd(hb, fx(c20 * r2b));
                if (c21 != 0.0f) atomicAdd(hb + NE2, fx(c21 * r2b));
            }
            if (r2a != 0.0f) {
                if (c22 != 0.0f) atomicAdd(hb + 2 * NE2, fx(c22 * r2a));
                if (c23 != 0.0f) atomicAdd(hb + 3 * NE2, fx(c23 * r2a));
            }
            r2a = 0.0f;
            r2b = 0.0f;
        };
        // one node of each class: p = Phi at the node's bin i, fa / fb = q f of
        // voxel j / of its mirror
        auto en_node = [&](uint32_t i1, float p1, uint32_t i2, float p2, float fa, float fb) {
            if (i1 != cur1) {
                flush1();
                cur1 = i1;
            }
            r1a = fmaf(p1, fa, r1a);
            if (LR) {
                r1b = fmaf(p1, fb, r1b);
                if (i2 != cur2) {
                    flush2();
                    cur2 = i2;
                }
                r2a = fmaf(p2, fa, r2a);
                r2b = fmaf(p2, fb, r2b);
            }
        };
        if (QU) {
            const double qa0 = P.a0 + P.da * m0;
            const double u10 = fma(k1, qa0, b0), du1 = k1 * P.da;
            const double u20 = fma(k2, qa0, b0), du2 = k2 * P.da;
            int lo = QW, hi = -1;
            if (ST) {
                // the (quad, tile) node range from the store: wave-uniform, a
                // superset of both classes' ranges over the lanes
                lo = (int)(tmeta & 0xffffu) - m0;
                hi = (int)(tmeta >> 16) - m0;
            } else {
                if (act1) band_range(P, u10, du1, 0, QW, lo, hi);
                if (LR && act2) {
                    int l2, h2;
                    band_range(P, u20, du2, 0, QW, l2, h2);
                    lo = min(lo, l2);
                    hi = max(hi, h2);
                }
            }
            constexpr int BF = ST ? QB_ST : (QB_FWD < QW ? QB_FWD : QW);
#pragma unroll
            for (int blk = 0; blk < QW / BF; ++blk) {
                // skip a block no lane of the wave has in band (its triples add exact zeros)
                if (ST) {
                    if (blk * BF + BF - 1 < lo || blk * BF > hi) continue;
                } else if (__ballot(lo <= blk * BF + BF - 1 && hi >= blk * BF) == 0) {
                    continue;
                }
                // anchored by an FMA at each block's first node, then one add per node
                double ua = fma((double)(blk * BF), du1, u10), ub = fma((double)(blk * BF), du2, u20);
#pragma unroll
                for (int mm = 0; mm < BF; ++mm) {
                    const int m = blk * BF + mm;
                    // the table's pads cover every coordinate: no clamp unless
                    // the bin keys an energy histogram
                    const int c1 = (int)ua;
                    const uint32_t i1 = min((uint32_t)c1, top);
                    const float p1 = EN ? spec(s_phi, i1) : s_phi[c1];
                    ua += du1;
                    if (LR) {
                        const int c2 = (int)ub;
                        const uint32_t i2 = min((uint32_t)c2, top);
                        const float p2 = EN ? spec(s_phi, i2) : s_phi[c2];
                        ub += du2;
                        const float2 fv = *(const float2 *)(trow + m * TS);
                        if (EN) {
                            en_node(i1, p1, i2, p2, fv.x, fv.y);
                        } else {
                            w1a = fmaf(p1, fv.x, w1a);
                            w1b = fmaf(p1, fv.y, w1b);
                            w2a = fmaf(p2, fv.x, w2a);
                            w2b = fmaf(p2, fv.y, w2b);
                        }
                    } else if (EN) {
                        en_node(i1, p1, 0u, 0.0f, trow[m * TS], 0.0f);
                    } else {
                        w1a = fmaf(p1, trow[m * TS], w1a);
                    }
                }
            }
        } else {
#pragma unroll
            for (int blk = 0; blk < NB; ++blk) {
                const double2 qr = qb_c[blk];
                const bool need = (act1 && k1 * qr.y >= P.band_lo && k1 * qr.x < P.band_hi) ||
                                  (act2 && k2 * qr.y >= P.band_lo && k2 * qr.x < P.band_hi);
                if (__ballot(need) == 0) continue;
#pragma unroll
                for (int mm = 0; mm < 8; ++mm) {
                    const int m = blk * 8 + mm;
                    const double am = qa_c[m];
                    const uint32_t i1 = spec_index(k1, am, b0, top);
                    const float p1 = spec(s_phi, i1);
                    if (LR) {
                        const uint32_t i2 = spec_index(k2, am, b0, top);
                        const float p2 = spec(s_phi, i2);
                        const float2 fv = *(const float2 *)(trow + m * TS);
                        if (EN) {
                            en_node(i1, p1, i2, p2, fv.x, fv.y);
                        } else {
                            w1a = fmaf(p1, fv.x, w1a);
                            w1b = fmaf(p1, fv.y, w1b);
                            w2a = fmaf(p2, fv.x, w2a);
                            w2b = fmaf(p2, fv.y, w2b);
                        }
                    } else if (EN) {
                        en_node(i1, p1, 0u, 0.0f, trow[m * TS], 0.0f);
                    } else {
                        w1a = fmaf(p1, trow[m * TS], w1a);
                    }
                }
            }
        }
        if (EN) {
            flush1();
            if (LR) flush2();
            continue;
        }
        o0 = fmaf(c10, w1a, o0);
        o1 = fmaf(c11, w1a, o1);
        if (LR) {
            o2 = fmaf(c12, w1b, o2);
            o3 = fmaf(c13, w1b, o3);
            o0 = fmaf(c20, w2b, o0);
            o1 = fmaf(c21, w2b, o1);
            o2 = fmaf(c22, w2a, o2);
            o3 = fmaf(c23, w2a, o3);
        }
        } while (0);
        if (DB) {
            if (t + 1 < t1) put_tile(s_tile + ((t + 1 - t0) & 1) * TBUF);
            __syncthreads();
        }
    }
    if (!wave_on) return;
    if (EN) {
        // the histograms' bins 1..ne to float: partial image [ne][npix]
        const double inv = sc[1];
        const bool bad = fx_scale == 0.0;       // non-finite input
        float *dst = part + (size_t)(by * gz + qc) * P.ne * P.npix;
        const int bd = P.ndy - 1 - bu, ab = P.ndx - 1 - a;
        const int px[4] = {bu * P.ndx + a, bd * P.ndx + a, bu * P.ndx + ab, bd * P.ndx + ab};
        for (int k = lane; k < P.ne; k += 64)
#pragma unroll
            for (int o = 0; o < (LR ? 4 : 2); ++o) {
                const long long v = (long long)hist[o * NE2 + k + 1];
                dst[(size_t)k * P.npix + px[o]] = bad ? __builtin_nanf("") : (float)((double)v * inv);
            }
        return;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        o0 += __shfl_xor(o0, off, 64);
        o1 += __shfl_xor(o1, off, 64);
        if (LR) {
            o2 += __shfl_xor(o2, off, 64);
            o3 += __shfl_xor(o3, off, 64);
        }
    }
    if (lane == 0) {
        float *dst = part + (size_t)(by * gz + qc) * P.npix;
        const int bd = P.ndy - 1 - bu;
        dst[bu * P.ndx + a] = o0;
        dst[bd * P.ndx + a] = o1;
        if (LR) {
            const int ab = P.ndx - 1 - a;
            dst[bu * P.ndx + ab] = o2;
            dst[bd * P.ndx + ab] = o3;
        }
    }
}

template <int LR, int QW, int QU, int ST>
__global__ void __launch_bounds__(256) k_adjoint(KParams P, DevTables T, Lds L,
                                                 const double *__restrict__ qa,
                                                 const double2 *__restrict__ qblk,
                                                 const float *__restrict__ rho,
                                                 float *__restrict__ b)
{
    adjoint_body<LR, QW, QU, 0, ST>(P, T, L, qa, qblk, rho, b, blockIdx.x, blockIdx.y, blockIdx.z);
}

template <int LR, int QW, int QU, int ST>
__global__ void __launch_bounds__(512) k_forward(KParams P, DevTables T, Lds L,
                                                 const double *__restrict__ qa,
                                                 const double2 *__restrict__ qblk,
                                                 const float *__restrict__ f,
                                                 float *__restrict__ part, int tiles_per_split)
{
    int bx, by, bz;
    xcd_block(bx, by, bz);
    forward_body<LR, QW, QU, 0, ST>(P, T, L, qa, qblk, f, part, tiles_per_split, bx, by, bz, gridDim.z);
}

// Global q-node range [lo, hi] of a class with Bragg factor kappa on a
// uniform grid: the nodes whose bin coordinate u_m = u0 + m du can lie in
// [1, ne + 1), with one node of margin each side (nodes outside add exact
// zeros, so a superset is always safe).  Empty (lo > hi) when inactive.
__device__ __forceinline__ void node_range(const KParams &P, bool active, double kappa, int &lo, int &hi)
{
    lo = 0xffff;
    hi = -1;
    if (!active) return;
    const double u0 = fma(kappa, P.a0, P.b0), du = kappa * P.da;
    const double a = floor((1.0 - u0) / du) - 1.0, b = floor(((double)P.ne + 1.0 - u0) / du) + 1.0;
    lo = (int)fmin(fmax(a, 0.0), (double)(P.nq - 1));
    hi = (int)fmin(fmax(b, 0.0), (double)(P.nq - 1));
}

// Tile record of the node ranges of a wave's 64 lanes (lane 0 writes).
__device__ __forceinline__ void write_tile_range(uint32_t *dst, int lo, int hi)
{
    lo = wave_min(lo);
    hi = wave_max(hi);
    if ((threadIdx.x & 63) == 0) *dst = lo > hi ? 0xffffu : ((uint32_t)lo | ((uint32_t)hi << 16));
}

// Factor store of the adjoint: the record of voxel group g and pixel class
// (a, r) in tile t, lane l -- kappa, A and the mask values exactly as
// adjoint_body evaluates them, A = kappa = 0 and no bits when the class is
// inactive (every pair closed, or kappa out of band).  One thread per record.
template <int LR>
__device__ __forceinline__ uint4 adjoint_record(const KParams &P, const DevTables &T, int g, int a, int r,
                                                double &k, uint32_t &bits)
{
    const int half_y = P.ndy / 2;
    int j = g;
    if (LR) {
        const int half = P.nx / 2;
        j = (g / half) * P.nx + g % half;
    }
    k = 0.0;
    float A = 0.0f;
    bits = 0u;
    if (a < P.ndx && r < half_y) {
        const int bu = half_y + r;
        const double xp = pixel_coord(P, a, P.ndx);
        const double yp = pixel_coord(P, bu, P.ndy);
        const Cells c = mask_cells(P, T.vm[j], xp, yp);
        if (c.in_rows) {
            const uint32_t ru = T.maskbits[c.row_u], rd = T.maskbits[c.row_d];
            bits = ((ru >> c.col_a) & 1u) | (((rd >> c.col_a) & 1u) << 1);
            if (LR) bits |= (((ru >> c.col_b) & 1u) << 2) | (((rd >> c.col_b) & 1u) << 3);
        }
        if (bits) {
            pair_factors(P, T.vd[j], T.vf[j], xp, yp, k, A);
            if (in_band(P, k)) {
                bits |= CSX_REC_ACT;
            } else {
                bits = 0u;
                k = 0.0;
                A = 0.0f;
            }
        }
    }
    const uint64_t ku = (uint64_t)__double_as_longlong(k);
    return make_uint4((uint32_t)ku, (uint32_t)(ku >> 32), __float_as_uint(A), bits);
}

template <int LR>
__global__ void __launch_bounds__(256) k_store_adjoint(KParams P, DevTables T, uint4 *__restrict__ out,
                                                       uint32_t *__restrict__ meta)
{
    const int half_y = P.ndy / 2, ntx = (P.ndx + 7) / 8;
    const int ntl = ntx * ((half_y + 7) / 8);
    const size_t idx = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (idx >= (size_t)P.n_groups * ntl * 64) return;
    const int g = (int)(idx / ((size_t)ntl * 64));
    const int e = (int)(idx % ((size_t)ntl * 64));
    const int t = e >> 6, lane = e & 63;
    const int a = (t % ntx) * 8 + (lane & 7), r = (t / ntx) * 8 + (lane >> 3);
    double k;
    uint32_t bits;
    out[idx] = adjoint_record<LR>(P, T, g, a, r, k, bits);
    int lo, hi;
    node_range(P, (bits & CSX_REC_ACT) != 0u, k, lo, hi);
    write_tile_range(meta + idx / 64, lo, hi);
}

// The same records in the order of class lists: list p of n_sub, n_cls
// classes each (class = r ndx + a), padded to cls_pad (a multiple of 64;
// the padding is inactive); record of (group g, list p, entry e) at
// (g n_sub + p) cls_pad + e, node range per 64 entries.  One thread per record.
template <int LR>
__global__ void __launch_bounds__(256) k_store_adjoint_list(KParams P, DevTables T, const int *__restrict__ cls,
                                                            int n_cls, int n_sub, int cls_pad,
                                                            uint4 *__restrict__ out, uint32_t *__restrict__ meta)
{
    const size_t idx = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (idx >= (size_t)P.n_groups * n_sub * cls_pad) return;
    const int g = (int)(idx / ((size_t)n_sub * cls_pad));
    const int rem = (int)(idx % ((size_t)n_sub * cls_pad));
    const int p = rem / cls_pad, e = rem % cls_pad;
    int a = P.ndx, r = P.ndy;                  // padding: outside the detector, inactive
    if (e < n_cls) {
        const int c = cls[(size_t)p * n_cls + e];
        a = c % P.ndx;
        r = c / P.ndx;
    }
    double k;
    uint32_t bits;
    out[idx] = adjoint_record<LR>(P, T, g, a, r, k, bits);
    int lo, hi;
    node_range(P, (bits & CSX_REC_ACT) != 0u, k, lo, hi);
    write_tile_range(meta + idx / 64, lo, hi);
}

// Factor store of the forward: for pixel quad qq and voxel group (tile t,
// lane l) the two classes of forward_body -- class 1 at pixel column a,
// class 2 at its mirror -a -- as two 16-byte words {kappa1, kappa2} and
// {A1, A2, bits, 0}.  One thread per (quad, group).
template <int LR>
__global__ void __launch_bounds__(256) k_store_forward(KParams P, DevTables T, uint4 *__restrict__ out,
                                                       uint32_t *__restrict__ meta)
{
    const int gw = LR ? P.nx / 2 : P.nx;
    const int ntx = (gw + 7) / 8;
    const int ntl = ntx * ((P.nz + 7) / 8);
    const size_t idx = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (idx >= (size_t)P.n_quad * ntl * 64) return;
    const int qq = (int)(idx / ((size_t)ntl * 64));
    const int e = (int)(idx % ((size_t)ntl * 64));
    const int t = e >> 6, lane = e & 63;
    int a, bu;
    if (LR) {
        const int hx = P.ndx / 2;
        a = hx + qq % hx;
        bu = P.ndy / 2 + qq / hx;
    } else {
        a = qq % P.ndx;
        bu = P.ndy / 2 + qq / P.ndx;
    }
    const double xpa = pixel_coord(P, a, P.ndx);
    const double yp = pixel_coord(P, bu, P.ndy);
    const int ix = (t % ntx) * 8 + (lane & 7), iz = (t / ntx) * 8 + (lane >> 3);
    double k1 = 0.0, k2 = 0.0;
    float A1 = 0.0f, A2 = 0.0f;
    uint32_t bits = 0u;
    if (ix < gw && iz < P.nz) {
        const int j = iz * P.nx + ix;
        const VoxD vd = T.vd[j];
        const float2 vf = T.vf[j];
        const double2 vm = T.vm[j];
        for (int cls = 0; cls < (LR ? 2 : 1); ++cls) {
            const double xp = cls ? -xpa : xpa;
            const Cells c = mask_cells(P, vm, xp, yp);
            uint32_t b = 0u;
            if (c.in_rows) {
                const uint32_t ru = T.maskbits[c.row_u], rd = T.maskbits[c.row_d];
                b = ((ru >> c.col_a) & 1u) | (((rd >> c.col_a) & 1u) << 1);
                if (LR) b |= (((ru >> c.col_b) & 1u) << 2) | (((rd >> c.col_b) & 1u) << 3);
            }
            if (b) {
                double k;
                float A;
                pair_factors(P, vd, vf, xp, yp, k, A);
                if (in_band(P, k)) {
                    bits |= (b | CSX_REC_ACT) << (8 * cls);
                    if (cls) {
                        k2 = k;
                        A2 = A;
                    } else {
                        k1 = k;
                        A1 = A;
                    }
                }
            }
        }
    }
    const uint64_t u1 = (uint64_t)__double_as_longlong(k1), u2 = (uint64_t)__double_as_longlong(k2);
    const size_t o = idx * 2;
    out[o] = make_uint4((uint32_t)u1, (uint32_t)(u1 >> 32), (uint32_t)u2, (uint32_t)(u2 >> 32));
    out[o + 1] = make_uint4(__float_as_uint(A1), __float_as_uint(A2), bits, 0u);
    int lo1, hi1, lo2, hi2;
    node_range(P, (bits & CSX_REC_ACT) != 0u, k1, lo1, hi1);
    node_range(P, (bits & (CSX_REC_ACT << 8)) != 0u, k2, lo2, hi2);
    write_tile_range(meta + idx / 64, min(lo1, lo2), max(hi1, hi2));
}

// Energy-resolved operators (the energy-sensitive detector of App. A).
template <int LR, int QW, int QU>
__global__ void __launch_bounds__(256) k_adjoint_energy(KParams P, DevTables T, Lds L,
                                                        const double *__restrict__ qa,
                                                        const double2 *__restrict__ qblk,
                                                        const float *__restrict__ psi,
                                                        float *__restrict__ b)
{
    adjoint_body<LR, QW, QU, 1>(P, T, L, qa, qblk, psi, b, blockIdx.x, blockIdx.y);
}

template <int LR, int QW, int QU>
__global__ void __launch_bounds__(512) k_forward_energy(KParams P, DevTables T, Lds L,
                                                        const double *__restrict__ qa,
                                                        const double2 *__restrict__ qblk,
                                                        const float *__restrict__ f,
                                                        float *__restrict__ part, int tiles_per_split,
                                                        const double *__restrict__ sc)
{
    int bx, by, bz;
    xcd_block(bx, by, bz);
    forward_body<LR, QW, QU, 1>(P, T, L, qa, qblk, f, part, tiles_per_split, bx, by, bz, gridDim.z, sc);
}

// Energy-resolved adjoint with the Phi-weighted data staged in LDS: a block
// of waves (one voxel group each: voxel j and, with LR, its mirror j2) walks
// the pixel-class tiles together; for each 8 x 8 tile of classes (a, upper
// row r) the block copies Psi[k][pixel] of the tile's pixels for every bin k
// into LDS, slot = set * 64 + lane with sets u = (bu, a), d = (bd, a) and,
// with LR, (bu, -a), (bd, -a); a lane then reads its class's pixel values at
// a triple's bin from LDS.
template <int LR, int QW, int QU>
__global__ void __launch_bounds__(LR ? 512 : 1024) k_adjoint_energy_tiled(KParams P, DevTables T, Lds L,
                                                               const double *__restrict__ qa,
                                                               const double2 *__restrict__ qblk,
                                                               const float *__restrict__ psi,
                                                               float *__restrict__ b)
{
    constexpr int NB = QW / 8;
    constexpr int NSET = LR ? 4 : 2;
    constexpr int SLOTS = 64 * NSET;
    extern __shared__ __align__(16) unsigned char lds[];
    uint32_t *s_bits = (uint32_t *)(lds + L.mask);
    float *s_psi = (float *)(lds + L.tile);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int k = threadIdx.x; k < P.mask_ny; k += blockDim.x) s_bits[k] = T.maskbits[k];
    const int NE2 = P.ne + 2;
    const int g = blockIdx.x * (blockDim.x >> 6) + wv;
    const bool von = g < P.n_groups;
    int j = 0, j2 = 0;
    if (von) {
        if (LR) {
            const int half = P.nx / 2;
            j = (g / half) * P.nx + g % half;
            j2 = (g / half) * P.nx + (P.nx - 1 - g % half);
        } else {
            j = g;
            j2 = g;
        }
    }
    VoxD vd = {0.0, 1.0, 1.0, 0.0};
    float2 vf = {0.0f, 0.0f};
    double2 vm = {0.0, 0.0};
    if (von) {
        vd = T.vd[j];
        vf = T.vf[j];
        vm = T.vm[j];
    }
    const int m0 = blockIdx.y * QW;
    const double *qa_c = qa + m0;
    const double2 *qb_c = qblk + blockIdx.y * NB;
    const double b0 = P.b0;
    const uint32_t top = (uint32_t)(P.ne + 1);
    float acc0[QW], acc1[QW];
#pragma unroll
    for (int m = 0; m < QW; ++m) {
        acc0[m] = 0.0f;
        acc1[m] = 0.0f;
    }
    const int half_y = P.ndy / 2;
    const int ntx = (P.ndx + 7) / 8;
    const int ntiles = ntx * ((half_y + 7) / 8);
    for (int t = 0; t < ntiles; ++t) {
        const int ta = (t % ntx) * 8, tr = (t / ntx) * 8;
        __syncthreads();
        // staging: thread = pixel slots slot0, slot0 + blockDim, ... and every bin
        for (int slot = threadIdx.x % SLOTS; slot < SLOTS; slot += blockDim.x) {
            const int c = slot & 63, set = slot >> 6;
            const int a = ta + (c & 7), r = tr + (c >> 3);
            const bool valid = a < P.ndx && r < half_y;
            const int bu = half_y + r;
            const int row = (set & 1) ? P.ndy - 1 - bu : bu;
            const int col = (set & 2) ? P.ndx - 1 - a : a;
            const float *src = psi + (valid ? row * P.ndx + col : 0);
            const int k0 = threadIdx.x / SLOTS, kstep = max(1, (int)blockDim.x / SLOTS);
            // unconditional loads (an invalid slot reads pixel 0 and stores 0),
            // two in flight at a time
#pragma unroll 2
            for (int k = k0; k < NE2; k += kstep) {
                const float v = src[(size_t)k * P.npix];
                s_psi[k * SLOTS + slot] = valid ? v : 0.0f;
            }
            if ((int)blockDim.x >= SLOTS) break;
        }
        __syncthreads();
        if (!von) continue;
        const int a = ta + (lane & 7), r = tr + (lane >> 3);
        double kap = 0.0;
        float eu = 0.0f, ed = 0.0f, ebu = 0.0f, ebd = 0.0f;
        bool act = false;
        if (a < P.ndx && r < half_y) {
            const int bu = half_y + r;
            const double xp = pixel_coord(P, a, P.ndx);
            const double yp = pixel_coord(P, bu, P.ndy);
            const Cells c = mask_cells(P, vm, xp, yp);
            if (c.in_rows) {
                const uint32_t ru = s_bits[c.row_u], rd = s_bits[c.row_d];
                const float tu = bitf(ru, c.col_a), td = bitf(rd, c.col_a);
                const float tbu = LR ? bitf(ru, c.col_b) : 0.0f, tbd = LR ? bitf(rd, c.col_b) : 0.0f;
                if (tu + td + tbu + tbd != 0.0f) {
                    double k;
                    float A;
                    pair_factors(P, vd, vf, xp, yp, k, A);
                    if (in_band(P, k)) {
                        eu = A * tu;
                        ed = A * td;
                        ebu = A * tbu;
                        ebd = A * tbd;
                        kap = k;
                        act = true;
                    }
                }
            }
        }
        if (__ballot(act) == 0) continue;
        const float *ps = s_psi + lane;
        auto node = [&](int m, uint32_t kk) {
            const float *row = ps + kk * SLOTS;
            acc0[m] = fmaf(eu, row[0], fmaf(ed, row[64], acc0[m]));
            if (LR) acc1[m] = fmaf(ebu, row[128], fmaf(ebd, row[192], acc1[m]));
        };
        if (QU) {
            const double u0 = fma(kap, P.a0 + P.da * m0, b0), du = kap * P.da;
            int lo = QW, hi = -1;
            if (act) band_range(P, u0, du, 0, QW, lo, hi);
#pragma unroll
            for (int blk = 0; blk < NB; ++blk) {
                // skip a block no lane of the wave has in band (its triples add exact zeros)
                if (__ballot(lo <= blk * 8 + 7 && hi >= blk * 8) == 0) continue;
                double u = fma((double)(blk * 8), du, u0);
#pragma unroll
                for (int mm = 0; mm < 8; ++mm) {
                    const uint32_t kk = min((uint32_t)(int)u, top);
                    u += du;
                    node(blk * 8 + mm, kk);
                }
            }
        } else {
#pragma unroll
            for (int blk = 0; blk < NB; ++blk) {
                const double2 qr = qb_c[blk];
                const bool need = act && kap * qr.y >= P.band_lo && kap * qr.x < P.band_hi;
                if (__ballot(need) == 0) continue;
#pragma unroll
                for (int mm = 0; mm < 8; ++mm) node(blk * 8 + mm, spec_index(kap, qa_c[blk * 8 + mm], b0, top));
            }
        }
    }
    if (!von) return;
    WaveTransposeSum<QW, 32>::run(acc0, lane);
    if (LR) WaveTransposeSum<QW, 32>::run(acc1, lane);
    const int mi = transposed_index<QW>(lane);
    const int m = m0 + mi;
    const bool writer = (lane & ((64 / QW) - 1)) == 0;
    if (writer && m < P.nq) {
        const float qm = T.qv[m];
        b[(size_t)j * P.nq + m] = acc0[0] * qm;
        if (LR) b[(size_t)j2 * P.nq + m] = acc1[0] * qm;
    }
}

// Batched launches: the blocks of several scans in one grid.  Block b belongs
// to the job whose [begin, begin + blocks) range holds it (binary search over
// the sorted begin offsets); its local index is decoded into that job's grid.
__device__ __forceinline__ int find_job(const int *__restrict__ begin, int njobs, int b)
{
    int lo = 0, hi = njobs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (begin[mid] <= b) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

template <int LR, int QW, int QU, int ST>
__global__ void __launch_bounds__(256) k_adjoint_batch(const CsxJob *__restrict__ jobs,
                                                       const int *__restrict__ begin, int njobs)
{
    const int jb = find_job(begin, njobs, blockIdx.x);
    const CsxJob &J = jobs[jb];
    const int local = blockIdx.x - begin[jb];
    adjoint_body<LR, QW, QU, 0, ST>(J.P, J.T, J.L, J.T.qa, J.T.qblk, J.in, J.out, local % J.gx,
                                        local / J.gx);
}

template <int LR, int QW, int QU, int ST>
__global__ void __launch_bounds__(512) k_forward_batch(const CsxJob *__restrict__ jobs,
                                                       const int *__restrict__ begin, int njobs)
{
    const int jb = find_job(begin, njobs, blockIdx.x);
    const CsxJob &J = jobs[jb];
    // within each job, the XCD-aware numbering of the single-scan forward: the
    // job's blocks on XCD x (= blockIdx.x mod 8, round-robin dispatch) take the
    // x-th eighth of its (quad group, q chunk, split) grid, split slowest
    int local = blockIdx.x - begin[jb];
    const int n = J.gx * J.gy * J.gz;
    if (n % 8 == 0) local = (int)(blockIdx.x % 8) * (n / 8) + local / 8;
    const int bx = local % J.gx, r = local / J.gx;
    forward_body<LR, QW, QU, 0, ST>(J.P, J.T, J.L, J.T.qa, J.T.qblk, J.in, J.out, J.tps, bx, r / J.gz,
                                        r % J.gz, J.gz);
}

// g_i = sum_p part[p][i] in a fixed order.
__global__ void __launch_bounds__(256) k_sum_parts(const float *__restrict__ part, int nparts, int n,
                                                   float *__restrict__ g)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float s = 0.0f;
    for (int p = 0; p < nparts; ++p) s += part[(size_t)p * n + i];
    g[i] = s;
}

// Subset forward, finished: at the listed pixels z = sum of the partial
// images (+ r) and rho = y / z (0 where y = 0 or z <= 0).  One wave per pixel:
// lane k adds partials k, k + 64, ..., then a fixed butterfly adds the lanes.
__global__ void __launch_bounds__(64) k_sum_ratio_list(const float *__restrict__ part, int nparts, int npix,
                                                      const int *__restrict__ pix, const float *__restrict__ y,
                                                      const float *__restrict__ r, float *__restrict__ rho)
{
    const int i = pix[blockIdx.x];
    const int lane = threadIdx.x;
    float s = 0.0f;
    for (int p = lane; p < nparts; p += 64) s += part[(size_t)p * npix + i];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    if (lane == 0) {
        const float z = s + (r ? r[i] : 0.0f);
        const float yi = y[i];
        rho[i] = (yi > 0.0f && z > 0.0f) ? yi / z : 0.0f;
    }
}

// LDS of an operator launch: spectrum table, mask bits and, for the forward,
// the q f tile (two buffers for the energy-integrating forward, one for the
// energy-resolved one).
Lds lds_layout(const KParams &P, bool forward, bool energy = false)
{
    auto al = [](int v) { return (v + 15) & ~15; };
    Lds L;
    int off = 0;
    L.phi = off;
    off += al(P.spec_n * 4);
    L.mask = off;
    off += al(P.mask_ny * 4);
    L.tile = off;
    if (forward) off += (energy ? 1 : 2) * P.qw * (64 * (P.lr ? 2 : 1) + 2) * 4;
    L.total = off;
    return L;
}

int fwd_tiles(const KParams &P)
{
    const int gw = P.lr ? P.nx / 2 : P.nx;
    return ((gw + 7) / 8) * ((P.nz + 7) / 8);
}

int log2i(int v)
{
    int r = 0;
    while ((1 << r) < v) ++r;
    return r;
}

// Kernel template of a launch: bit 0 factor store, bit 1 LR mirror, bit 2
// uniform q, bits 3+ log2 of the q chunk width.  (The table dtype only
// changes table staging.)
int variant_of(const KParams &P, bool stored = false)
{
    return (stored && P.qu ? 1 : 0) | (P.lr ? 2 : 0) | (P.qu ? 4 : 0) | (log2i(P.qw) << 3);
}

// Template dispatch: variant -> kernel instance (the factor store exists on
// uniform q grids only).
template <template <int, int, int, int> class K, typename... A>
void dispatch(int variant, A &&...a)
{
    const int st = variant & 1, lr = (variant >> 1) & 1, qu = (variant >> 2) & 1;
    const int qw = 1 << (variant >> 3);
#define CSX_CASE(LR_, QW_, QU_, ST_) \
    if (lr == LR_ && qw == QW_ && qu == QU_ && st == ST_) { K<LR_, QW_, QU_, ST_>::run(a...); return; }
#define CSX_CASES_QW(LR_, QU_, ST_) CSX_CASE(LR_, 16, QU_, ST_) CSX_CASE(LR_, 32, QU_, ST_) CSX_CASE(LR_, 64, QU_, ST_)
    CSX_CASES_QW(0, 0, 0) CSX_CASES_QW(0, 1, 0) CSX_CASES_QW(1, 0, 0) CSX_CASES_QW(1, 1, 0)
    CSX_CASES_QW(0, 1, 1) CSX_CASES_QW(1, 1, 1)
#undef CSX_CASES_QW
#undef CSX_CASE
}

template <int LR, int QW, int QU, int ST>
struct RunFwd {
    static void run(const OpShape &S, const csx_geometry *h, const float *f, float *part, hipStream_t s)
    {
        hipLaunchKernelGGL((k_forward<LR, QW, QU, ST>), S.grid, S.block, S.L.total, s, S.P, h->t,
                           S.L, h->t.qa, h->t.qblk, f, part, S.tps);
    }
};

template <int LR, int QW, int QU, int ST>
struct RunAdj {
    static void run(const OpShape &S, const csx_geometry *h, const float *rho, float *b,
                    hipStream_t s)
    {
        const DevTables &T = S.T ? *S.T : h->t;
        hipLaunchKernelGGL((k_adjoint<LR, QW, QU, ST>), S.grid, S.block, S.L.total, s, S.P, T,
                           S.L, T.qa, T.qblk, rho, b);
    }
};

template <int LR, int QW, int QU, int ST>
struct RunFwdBatch {
    static void run(const CsxJob *jobs, const int *begin, int njobs, int nblocks, int lds,
                    hipStream_t s)
    {
        hipLaunchKernelGGL((k_forward_batch<LR, QW, QU, ST>), dim3(nblocks), dim3(512), lds, s,
                           jobs, begin, njobs);
    }
};

template <int LR, int QW, int QU, int ST>
struct RunAdjBatch {
    static void run(const CsxJob *jobs, const int *begin, int njobs, int nblocks, int lds,
                    hipStream_t s)
    {
        hipLaunchKernelGGL((k_adjoint_batch<LR, QW, QU, ST>), dim3(nblocks), dim3(256), lds, s,
                           jobs, begin, njobs);
    }
};

template <int LR, int QW, int QU, int ST>
struct RunFwdE {
    static void run(const OpShape &S, const csx_geometry *h, const float *f, float *part, const double *sc,
                    hipStream_t s)
    {
        if constexpr (ST == 0)
            hipLaunchKernelGGL((k_forward_energy<LR, QW, QU>), S.grid, S.block, S.L.total, s, S.P, h->t, S.L,
                               h->t.qa, h->t.qblk, f, part, S.tps, sc);
    }
};

template <int LR, int QW, int QU, int ST>
struct RunAdjE {
    static void run(const OpShape &S, const csx_geometry *h, const float *psi, float *b, hipStream_t s)
    {
        if constexpr (ST == 0)
            hipLaunchKernelGGL((k_adjoint_energy<LR, QW, QU>), S.grid, S.block, S.L.total, s, S.P, h->t, S.L,
                               h->t.qa, h->t.qblk, psi, b);
    }
};

// Launch shape of the energy-resolved forward: the widest q chunk whose LDS
// (q f tile plus the 8 waves' histograms) fits, and enough voxel splits for
// ~2048 blocks.
OpShape forward_energy_shape(const csx_geometry *h)
{
    OpShape S;
    S.P = h->P;
    S.P.qw = S.P.nq <= 16 ? 16 : (S.P.nq <= 32 ? 32 : 64);
    auto lay = [&]() {
        S.P.qchunks = (S.P.nq + S.P.qw - 1) / S.P.qw;
        S.L = lds_layout(S.P, true, true);
        S.L.hist = (S.L.total + 15) & ~15;
        S.L.total = S.L.hist + 8 * 4 * (S.P.ne + 2) * 8;
    };
    lay();
    while (S.L.total > CSX_LDS_MAX && S.P.qw > 16) {   // narrower q chunks leave room for the histograms
        S.P.qw /= 2;
        lay();
    }
    const int ntiles = fwd_tiles(S.P);
    const int bx = (S.P.n_quad + 7) / 8;
    const int splits = std::max(1, std::min(std::min(16, ntiles), 2048 / std::max(1, bx * S.P.qchunks)));
    S.tps = (ntiles + splits - 1) / splits;
    const int nsplit = (ntiles + S.tps - 1) / S.tps;
    S.grid = dim3(bx, nsplit, S.P.qchunks);
    S.block = dim3(512);
    S.nparts = nsplit * S.P.qchunks;
    S.variant = variant_of(S.P);
    return S;
}

}  // namespace

size_t csx_forward_energy_floats(const csx_geometry *h, int *lds_bytes)
{
    const OpShape S = forward_energy_shape(h);
    if (lds_bytes) *lds_bytes = S.L.total;
    return (size_t)S.nparts * h->P.ne * h->P.npix;
}

csx_status csx_launch_forward_energy(csx_geometry *h, const float *f, const double *sc, float *part,
                                     size_t part_cap, float *gE, hipStream_t s)
{
    const OpShape S = forward_energy_shape(h);
    const size_t n = (size_t)h->P.ne * h->P.npix;
    if ((size_t)S.nparts * n > part_cap) return csx_fail(CSX_EINVAL, "energy partials too small");
    if (S.L.total > CSX_LDS_MAX) return csx_fail(CSX_EINVAL, "energy-resolved forward: ne too large for LDS");
    dispatch<RunFwdE>(S.variant, S, h, f, part, sc, s);
    HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(k_sum_parts, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, part, S.nparts, (int)n, gE);
    HIP_TRY(hipGetLastError());
    return CSX_OK;
}

csx_status csx_launch_adjoint_energy(csx_geometry *h, const float *psi, float *b, hipStream_t s)
{
    {   // staged form when a tile of Psi fits in LDS (gfx950: up to 160 KiB per block)
        KParams P = h->P;
        P.qw = P.nq <= 16 ? 16 : 32;   // (64-q chunks measured no faster: 2 waves / SIMD)
        P.qchunks = (P.nq + P.qw - 1) / P.qw;
        auto layout = [&](int nset) {
            Lds L;
            L.phi = 0;
            L.mask = 0;
            L.tile = ((P.mask_ny * 4) + 15) & ~15;
            L.total = L.tile + (P.ne + 2) * 64 * nset * 4;
            return L;
        };
        const bool lr = P.lr && layout(4).total <= CSX_LDS_MAX;
        const Lds L = layout(lr ? 4 : 2);
        if (L.total <= CSX_LDS_MAX) {
            const int wpb = lr ? 8 : 16;      // waves per block (VGPRs: LR keeps two accumulator sets)
            const int groups = lr ? P.n_groups : P.nvox;
            if (!lr) {
                P.lr = 0;
                P.n_groups = P.nvox;
            }
            const dim3 grid((groups + wpb - 1) / wpb, P.qchunks);
            const dim3 block(64 * wpb);
#define CSX_EA(LR_, QW_, QU_) \
    hipLaunchKernelGGL((k_adjoint_energy_tiled<LR_, QW_, QU_>), grid, block, L.total, s, P, h->t, L, h->t.qa, \
                       h->t.qblk, psi, b)
            if (lr) {
                if (P.qw == 16) { if (P.qu) CSX_EA(1, 16, 1); else CSX_EA(1, 16, 0); }
                else { if (P.qu) CSX_EA(1, 32, 1); else CSX_EA(1, 32, 0); }
            } else {
                if (P.qw == 16) { if (P.qu) CSX_EA(0, 16, 1); else CSX_EA(0, 16, 0); }
                else { if (P.qu) CSX_EA(0, 32, 1); else CSX_EA(0, 32, 0); }
            }
#undef CSX_EA
            HIP_TRY(hipGetLastError());
            return CSX_OK;
        }
    }
    // q chunks of <= 32: the per-node gathers of Psi want more waves in flight
    // than the 64-wide accumulators of the energy-integrating adjoint allow
    OpShape S = csx_adjoint_shape(h);
    if (S.P.qw > 32) {
        S.P.qw = 32;
        S.P.qchunks = (S.P.nq + 31) / 32;
        S.grid.y = S.P.qchunks;
    }
    S.variant = variant_of(S.P);        // factors evaluated on the fly
    dispatch<RunAdjE>(S.variant, S, h, psi, b, s);
    HIP_TRY(hipGetLastError());
    return CSX_OK;
}

void csx_store_records(const KParams &P, size_t *n_adj, size_t *n_fwd)
{
    const int half_y = P.ndy / 2;
    const size_t adj_tiles = (size_t)((P.ndx + 7) / 8) * ((half_y + 7) / 8);
    *n_adj = (size_t)P.n_groups * adj_tiles * 64;
    *n_fwd = (size_t)P.n_quad * fwd_tiles(P) * 64;
}

csx_status csx_launch_store(const csx_geometry *h, uint4 *ra, uint4 *rf, uint32_t *ram, uint32_t *rfm,
                            hipStream_t s)
{
    size_t na, nf;
    csx_store_records(h->P, &na, &nf);
    const dim3 ga((unsigned)((na + 255) / 256)), gf((unsigned)((nf + 255) / 256));
    if (h->P.lr) {
        hipLaunchKernelGGL(k_store_adjoint<1>, ga, dim3(256), 0, s, h->P, h->t, ra, ram);
        hipLaunchKernelGGL(k_store_forward<1>, gf, dim3(256), 0, s, h->P, h->t, rf, rfm);
    } else {
        hipLaunchKernelGGL(k_store_adjoint<0>, ga, dim3(256), 0, s, h->P, h->t, ra, ram);
        hipLaunchKernelGGL(k_store_forward<0>, gf, dim3(256), 0, s, h->P, h->t, rf, rfm);
    }
    HIP_TRY(hipGetLastError());
    return CSX_OK;
}

csx_status csx_launch_store_list(const csx_geometry *h, const int *cls, int n_cls, int n_sub, int cls_pad, uint4 *out,
                                 uint32_t *meta, hipStream_t s)
{
    const size_t n = (size_t)h->P.n_groups * n_sub * cls_pad;
    const dim3 g((unsigned)((n + 255) / 256));
    if (h->P.lr)
        hipLaunchKernelGGL(k_store_adjoint_list<1>, g, dim3(256), 0, s, h->P, h->t, cls, n_cls, n_sub, cls_pad, out,
                           meta);
    else
        hipLaunchKernelGGL(k_store_adjoint_list<0>, g, dim3(256), 0, s, h->P, h->t, cls, n_cls, n_sub, cls_pad, out,
                           meta);
    HIP_TRY(hipGetLastError());
    return CSX_OK;
}

hipEvent_t csx_timing_event(csx_geometry *h, int op)
{
    if (!h->timing) return nullptr;
    std::vector<hipEvent_t> &v = h->ev[op];
    if (h->ev_used[op] == (int)v.size()) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        v.push_back(e);
    }
    return v[h->ev_used[op]++];
}

// Default tile ranges of the direct adjoint: enough for about 4 waves per
// SIMD (one wave per voxel group, q chunk and range), each range at least 4
// tiles of 64 classes.
int csx_default_adj_splits(const KParams &P, int adj_qw)
{
    const long qchunks = (P.nq + adj_qw - 1) / adj_qw;
    const long waves = std::max(1L, (long)P.n_groups * qchunks);
    const long ntiles = (long)((P.ndx + 7) / 8) * ((P.ndy / 2 + 7) / 8);
    // a launch of fewer than ~4 waves per SIMD (few voxel groups, e.g. the
    // paper's 28^2 voxels) is split to ~12: its waves are long (many class
    // tiles each), so more of them in flight hide their latencies
    if (waves >= 4L * 4 * 256) return 1;
    long sp = (12L * 4 * 256 + waves - 1) / waves;
    sp = std::min(sp, std::max(1L, ntiles / 4));
    return (int)std::max(1L, std::min(sp, 64L));
}

csx_launch csx_default_launch(const KParams &P)
{
    csx_launch lc;
    const int qw = P.nq <= 16 ? 16 : (P.nq <= 32 ? 32 : 64);
    lc.adj_qw = qw;
    // the forward's q chunk: narrower when its two q f tiles beside a long
    // spectrum table would leave room for only one 512-thread block per
    // compute unit
    int fq = qw;
    while (fq > 16) {
        KParams Q = P;
        Q.qw = fq;
        if (lds_layout(Q, true).total <= CSX_LDS_MAX / 2) break;
        fq /= 2;
    }
    lc.fwd_qw = fq;
    const int qchunks = (P.nq + fq - 1) / fq;
    // split the voxel tiles so that a forward launch holds >= ~8 waves per SIMD,
    // and, when f is larger than 1 MB, into at least 8 ranges: with the
    // XCD-aware block numbering each XCD then reads one eighth of f into its L2
    const int bx = (P.n_quad + 7) / 8;
    const int target_waves = 8 * 4 * 256;
    const int min_splits = (long)P.nvox * P.nq * 4 > (1L << 20) ? 8 : 1;
    int splits = std::max(min_splits, target_waves / std::max(1, bx * 8 * qchunks));
    splits = std::min(splits, std::max(1, fwd_tiles(P) / 2));
    lc.fwd_splits = std::min(splits, 64);
    lc.adj_splits = csx_default_adj_splits(P, lc.adj_qw);
    return lc;
}

bool csx_launch_valid(const csx_launch &lc)
{
    auto okq = [](int q) { return q == 16 || q == 32 || q == 64; };
    return okq(lc.fwd_qw) && okq(lc.adj_qw) && lc.fwd_splits >= 1 && lc.fwd_splits <= 64 && lc.adj_splits >= 1 &&
           lc.adj_splits <= 64;
}

OpShape csx_forward_shape(const csx_geometry *h)
{
    OpShape S;
    S.P = h->P;
    S.P.qw = h->lc.fwd_qw;
    S.P.qchunks = (S.P.nq + S.P.qw - 1) / S.P.qw;
    S.L = lds_layout(S.P, true);
    const int ntiles = fwd_tiles(S.P);
    const int splits = std::max(1, std::min(h->lc.fwd_splits, ntiles));
    S.tps = (ntiles + splits - 1) / splits;
    const int nsplit = (ntiles + S.tps - 1) / S.tps;
    S.grid = dim3((S.P.n_quad + 7) / 8, nsplit, S.P.qchunks);
    S.block = dim3(512);
    S.nparts = nsplit * S.P.qchunks;
    S.variant = variant_of(S.P, h->t.rf != nullptr);
    return S;
}

OpShape csx_adjoint_shape(const csx_geometry *h)
{
    OpShape S;
    S.P = h->P;
    S.P.qw = h->lc.adj_qw;
    S.P.qchunks = (S.P.nq + S.P.qw - 1) / S.P.qw;
    S.L = lds_layout(S.P, false);
    S.grid = dim3((S.P.n_groups + h->adj_wpb - 1) / h->adj_wpb, S.P.qchunks);
    S.block = dim3(64 * h->adj_wpb);
    S.tps = 0;
    S.nparts = 0;
    S.variant = variant_of(S.P, h->t.ra != nullptr);
    return S;
}

csx_status csx_launch_sum_parts(csx_geometry *h, int nparts, float *g, hipStream_t s)
{
    hipLaunchKernelGGL(k_sum_parts, dim3((h->P.npix + 255) / 256), dim3(256), 0, s, h->part,
                       nparts, h->P.npix, g);
    HIP_TRY(hipGetLastError());
    return CSX_OK;
}

csx_status csx_launch_forward(csx_geometry *h, const float *f, float *g, hipStream_t s)
{
    hipEvent_t e0 = csx_timing_event(h, 0), e1 = csx_timing_event(h, 0);
    if (e0) HIP_TRY(hipEventRecord(e0, s));
    if (h->iv) {
        csx_status st = csx_iv_forward(h, f, nullptr, 0, g, s);
        if (st != CSX_OK) return st;
    } else {
        const OpShape S = csx_forward_shape(h);
        dispatch<RunFwd>(S.variant, S, h, f, h->part, s);
        HIP_TRY(hipGetLastError());
        csx_status st = csx_launch_sum_parts(h, S.nparts, g, s);
        if (st != CSX_OK) return st;
    }
    if (e1) HIP_TRY(hipEventRecord(e1, s));
    return CSX_OK;
}

csx_status csx_launch_forward_parts(const csx_geometry *h, const float *f, float *part, size_t part_cap, float *g,
                                    hipStream_t s)
{
    if (h->iv) return csx_iv_forward(h, f, part, part_cap, g, s);
    const OpShape S = csx_forward_shape(h);
    if ((size_t)S.nparts * h->P.npix > part_cap) return csx_fail(CSX_EINVAL, "forward partials exceed the buffer");
    dispatch<RunFwd>(S.variant, S, h, f, part, s);
    HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(k_sum_parts, dim3((h->P.npix + 255) / 256), dim3(256), 0, s, (const float *)part,
                       S.nparts, h->P.npix, g);
    HIP_TRY(hipGetLastError());
    return CSX_OK;
}

csx_status csx_launch_adjoint(csx_geometry *h, const float *rho, float *b, hipStream_t s)
{
    hipEvent_t e0 = csx_timing_event(h, 1), e1 = csx_timing_event(h, 1);
    if (e0) HIP_TRY(hipEventRecord(e0, s));
    if (h->iv) {
        csx_status st = csx_iv_adjoint(h, rho, b, s);
        if (st != CSX_OK) return st;
    } else {
        OpShape S = csx_adjoint_shape(h);
        const int sp = h->lc.adj_splits;
        if (sp > 1 && (size_t)sp * h->P.nvox * h->P.nq <= h->apart_cap) {
            // tile ranges into partial images, added in range order
            S.P.asplit = sp;
            S.grid.z = sp;
            dispatch<RunAdj>(S.variant, S, h, rho, h->apart, s);
            const int n = h->P.nvox * h->P.nq;
            hipLaunchKernelGGL(k_sum_parts, dim3((n + 255) / 256), dim3(256), 0, s, (const float *)h->apart, sp, n,
                               b);
        } else {
            dispatch<RunAdj>(S.variant, S, h, rho, b, s);
        }
        HIP_TRY(hipGetLastError());
    }
    if (e1) HIP_TRY(hipEventRecord(e1, s));
    return CSX_OK;
}

OpShape csx_forward_shape_list(const csx_geometry *h, const int *quads, int n_quads, int splits)
{
    OpShape S = csx_forward_shape(h);
    S.P.quad_list = quads;
    S.P.n_quad = n_quads;
    const int ntiles = fwd_tiles(S.P);
    const int sp = std::max(1, std::min(splits, ntiles));
    S.tps = (ntiles + sp - 1) / sp;
    const int nsplit = (ntiles + S.tps - 1) / S.tps;
    S.grid = dim3((n_quads + 7) / 8, nsplit, S.P.qchunks);
    S.nparts = nsplit * S.P.qchunks;
    return S;
}

csx_status csx_launch_forward_list(csx_geometry *h, const float *f, const int *quads, int n_quads, int splits,
                                   const int *pix, int n_pix, const float *y, const float *r, float *rho,
                                   hipStream_t s)
{
    const OpShape S = csx_forward_shape_list(h, quads, n_quads, splits);
    if ((size_t)S.nparts * h->P.npix > h->part_cap) return csx_fail(CSX_EINVAL, "forward partials too small");
    dispatch<RunFwd>(S.variant, S, h, f, h->part, s);
    hipLaunchKernelGGL(k_sum_ratio_list, dim3(n_pix), dim3(64), 0, s, h->part, S.nparts, h->P.npix, pix, y, r,
                       rho);
    HIP_TRY(hipGetLastError());
    return CSX_OK;
}

csx_status csx_launch_sum_ratio_list(csx_geometry *h, int nparts, const int *pix, int n_pix, const float *y,
                                     const float *r, float *rho, hipStream_t s)
{
    hipLaunchKernelGGL(k_sum_ratio_list, dim3(n_pix), dim3(64), 0, s, h->part, nparts, h->P.npix, pix, y, r, rho);
    HIP_TRY(hipGetLastError());
    return CSX_OK;
}

csx_status csx_launch_adjoint_list(csx_geometry *h, const float *rho, const int *cls, int n_cls, float *b,
                                   hipStream_t s, const uint4 *ra_list, const uint32_t *ram_list, long ra_gs)
{
    OpShape S = csx_adjoint_shape(h);
    S.P.cls_list = cls;
    S.P.n_cls = n_cls;
    DevTables T = h->t;
    if (ra_list && h->t.ra) {
        // the factor store in this list's order
        T.ra = const_cast<uint4 *>(ra_list);
        T.ram = const_cast<uint32_t *>(ram_list);
        S.P.ra_gs = ra_gs;
        S.T = &T;
    }
    // a short class list (an ordered subset) gives each wave only a few
    // tiles: when the pair factors are evaluated, 32-wide q chunks halve the
    // per-wave reduction and the accumulator registers, which outweighs
    // evaluating each class twice; with the store in list order, reading a
    // record twice costs more than the wider reduction (the q sums are the
    // same whatever the chunking)
    if (S.P.qw == 64 && n_cls <= 4 * 64 && !(ra_list && h->t.ra)) {
        S.P.qw = 32;
        S.P.qchunks = (S.P.nq + 31) / 32;
        S.grid.y = S.P.qchunks;
        S.variant = variant_of(S.P, h->t.ra != nullptr);
    }
    dispatch<RunAdj>(S.variant, S, h, rho, b, s);
    HIP_TRY(hipGetLastError());
    return CSX_OK;
}

csx_status csx_launch_forward_batch(const CsxJob *jobs_dev, const int *begin_dev, int njobs,
                                    int nblocks, int variant, int lds_bytes, hipStream_t s)
{
    dispatch<RunFwdBatch>(variant, jobs_dev, begin_dev, njobs, nblocks, lds_bytes, s);
    HIP_TRY(hipGetLastError());
    return CSX_OK;
}

csx_status csx_launch_adjoint_batch(const CsxJob *jobs_dev, const int *begin_dev, int njobs,
                                    int nblocks, int variant, int lds_bytes, hipStream_t s)
{
    dispatch<RunAdjBatch>(variant, jobs_dev, begin_dev, njobs, nblocks, lds_bytes, s);
    HIP_TRY(hipGetLastError());
    return CSX_OK;
}
