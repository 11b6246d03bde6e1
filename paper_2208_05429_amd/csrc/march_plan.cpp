// march_plan.cpp -- the layout and launch of an in-place marching pass
// (march_plan.hpp).
#include "march_plan.hpp"

#include <algorithm>

#include "march_dispatch.hpp"
#include "march_sets.hpp"

namespace lbm {

bool march_shape_of(int storage, int M, int variant, int nz, bool plain, MarchPlan* r, int lat)
{
    if (lat != 19) {
        // D3Q15 / D3Q27: shapes by storage, variant and step count
        if (M > 2) return false;
        for (const SetShapes& e : kSetShapes)
            if (e.lat == lat && e.storage == storage && e.variant == variant) {
                const ShapeEntry& t = M == 2 ? e.m2 : e.m1;
                r->TY = t.TY;
                r->TZ = t.TZ;
                r->NT = t.NT;
                r->pr = t.pr;
                r->pf = 1;
                if (t.pr && ((nz % 2) != 0 || plain)) {
                    // pairs need an even row: the plain layout of the same tile
                    for (const SetShapes& o : kSetShapes) {
                        const ShapeEntry& u = M == 2 ? o.m2 : o.m1;
                        if (o.lat == lat && o.storage == storage && !u.pr && u.TY == t.TY && u.TZ == t.TZ) {
                            r->NT = u.NT;
                            r->pr = 0;
                            return true;
                        }
                    }
                    return false;
                }
                return true;
            }
        return false;
    }
    if (M == 3) {
        // three merged steps: the plain layout, FP32 storage (variant v takes entry v)
        const int n3 = int(sizeof(kShapesM3F32) / sizeof(ShapeEntry));
        if (storage != LBM_F32 || variant < 0 || variant >= n3) return false;
        r->TY = kShapesM3F32[variant].TY;
        r->TZ = kShapesM3F32[variant].TZ;
        r->NT = kShapesM3F32[variant].NT;
        r->pr = 0;
        r->pf = 1;
        return true;
    }
    const ShapeEntry* tab = storage == LBM_F64 ? kShapesF64 : kShapesF32;
    const int n = storage == LBM_F64 ? int(sizeof(kShapesF64) / sizeof(ShapeEntry))
                                     : int(sizeof(kShapesF32) / sizeof(ShapeEntry));
    int idx = 2 * variant + (M == 2 ? 0 : 1);
    if (variant < 0 || idx >= n || tab[idx].M != M) return false;
    // pairs of z-adjacent cells need an even row length: take the plain-layout
    // entry of the same tile (or else the first plain entry) for odd nz, and
    // where the caller asks for the plain layout
    if (tab[idx].pr && ((nz % 2) != 0 || plain)) {
        int alt = -1;
        for (int j = 0; j < n && alt < 0; ++j)
            if (!tab[j].pr && tab[j].M == M && tab[j].TY == tab[idx].TY && tab[j].TZ == tab[idx].TZ) alt = j;
        for (int j = 0; j < n && alt < 0; ++j)
            if (!tab[j].pr && tab[j].M == M) alt = j;
        if (alt < 0) return false;
        idx = alt;
    }
    r->TY = tab[idx].TY;
    r->TZ = tab[idx].TZ;
    r->NT = tab[idx].NT;
    r->pr = tab[idx].pr;
    r->pf = tab[idx].pf;
    return true;
}

// A plain-layout shape for M steps whose last tile row across a periodic y
// seam is at least as thick as the halo (or whole), in table order.
bool plain_shape_for_seam(int storage, int M, int ny, MarchPlan* r, int lat)
{
    if (lat != 19) {
        if (M > 2) return false;
        for (const SetShapes& e : kSetShapes) {
            const ShapeEntry& t = M == 2 ? e.m2 : e.m1;
            if (e.lat != lat || e.storage != storage || t.pr) continue;
            const int rem = ny % t.TY;
            if (rem != 0 && rem < M) continue;
            r->TY = t.TY;
            r->TZ = t.TZ;
            r->NT = t.NT;
            r->pr = 0;
            r->pf = 1;
            return true;
        }
        return false;
    }
    if (M == 3 && storage != LBM_F32) return false;
    const ShapeEntry* tab = M == 3 ? kShapesM3F32 : (storage == LBM_F64 ? kShapesF64 : kShapesF32);
    const int n = M == 3 ? int(sizeof(kShapesM3F32) / sizeof(ShapeEntry))
                         : (storage == LBM_F64 ? int(sizeof(kShapesF64) / sizeof(ShapeEntry))
                                               : int(sizeof(kShapesF32) / sizeof(ShapeEntry)));
    for (int j = 0; j < n; ++j) {
        if (tab[j].pr || tab[j].M != M) continue;
        const int rem = ny % tab[j].TY;
        if (rem != 0 && rem < M) continue;
        r->TY = tab[j].TY;
        r->TZ = tab[j].TZ;
        r->NT = tab[j].NT;
        r->pr = 0;
        r->pf = tab[j].pf;
        return true;
    }
    return false;
}

// Tiles, segments and the hazard neighbourhood of one marching pass.
lbm_status make_plan(const lbm_config& c, int M, int cap, MarchPlan* p, std::string* why, bool last_segments)
{
    MarchPlan r;
    r.M = M;
    const int lat = lat_of(c);
    if (!march_shape_of(c.storage, M, c.variant, c.nz, false, &r, lat))
        return fail(why, LBM_EUNSUPPORTED, "no compiled marching kernel for this storage/variant");
    const bool py = c.face[2] == LBM_PERIODIC, pz = c.face[4] == LBM_PERIODIC;
    r.nty = (c.ny + r.TY - 1) / r.TY;
    r.ntz = (c.nz + r.TZ - 1) / r.TZ;
    if (r.pr && r.nty * r.ntz > cap && py && c.ny % r.TY != 0) {
        // The pair-and-ring layout reads saved rows across a periodic y seam
        // only above a whole tile row; the plain layout of the same tile also
        // takes a ragged last row (if it is at least as thick as the halo).
        MarchPlan q = r;
        if (march_shape_of(c.storage, M, c.variant, c.nz, true, &q, lat)) {
            r = q;
            r.nty = (c.ny + r.TY - 1) / r.TY;
            r.ntz = (c.nz + r.TZ - 1) / r.TZ;
        }
    }
    if (!r.pr && r.nty * r.ntz > cap && py && c.ny % r.TY != 0 && c.ny % r.TY < M) {
        // that last row would be thinner than the halo: another plain tile
        // height may leave a thick enough one
        MarchPlan q = r;
        if (plain_shape_for_seam(c.storage, M, c.ny, &q, lat)) {
            r = q;
            r.nty = (c.ny + r.TY - 1) / r.TY;
            r.ntz = (c.nz + r.TZ - 1) / r.TZ;
        }
    }
    const int tiles = r.nty * r.ntz;
    r.nbands = 1;
    r.nty_band = r.nty;
    if (tiles > cap) {
        // rounds over bands of tile rows, each band's boundary rows saved first
        auto need = [&]() {
            return "the y-z plane needs " + std::to_string(tiles) +
                   " marching workgroups, more than can be co-resident (" + std::to_string(cap) + ")";
        };
        if (r.ntz > cap) return fail(why, LBM_EUNSUPPORTED, need() + ", even for one row of tiles");
        // Across the periodic y seam the last row of tiles reads the first
        // band's saved rows.  The pair-and-ring layout reads them only in the
        // ring rows above a whole tile; the plain layout in any frame row, but
        // only the last row of tiles may reach across the seam.
        if (py && c.ny % r.TY != 0 && (r.pr || c.ny % r.TY < M))
            return fail(why, LBM_EUNSUPPORTED,
                        need() + (r.pr ? "; rounds on a periodic y axis need whole tile rows"
                                     : "; rounds on a periodic y axis need a last row of tiles at least as thick as the halo"));
        r.nty_band = cap / r.ntz;
        r.nbands = (r.nty + r.nty_band - 1) / r.nty_band;
        if (c.ny - (r.nbands - 1) * r.nty_band * r.TY < M)
            return fail(why, LBM_EUNSUPPORTED, need() + "; the last band of rows is thinner than the halo");
    }
    const int tiles_run = r.nty_band * r.ntz;  // work items of one round, per segment
    // a periodic axis whose last tile is thinner than M lets halos reach two tiles away
    r.ry = (py && r.nty > 1 && c.ny % r.TY != 0 && c.ny % r.TY < M) ? 2 : 1;
    r.rz = (pz && r.ntz > 1 && c.nz % r.TZ != 0 && c.nz % r.TZ < M) ? 2 : 1;
    // x segments: as many as fit, each at least 2M planes long.  A segment
    // marches seg_len + 2M planes; where the lattice is small the march is
    // bound by the latency of each plane, not by bytes, so short segments
    // pay for their re-read halo planes (128 x 64 x 64: 20 % less time per
    // step than segments of 4M planes; larger lattices run out of workgroups
    // first).  Neighbouring segments guard each other only, which needs
    // seg_len >= M.
    auto split = [&](int items, int* nseg_out, int* len_out) {
        int nseg = cap / items;
        const int by_len = c.nx / (2 * M);
        if (nseg > by_len) nseg = by_len;
        if (nseg < 1) nseg = 1;
        int seg_len = (c.nx + nseg - 1) / nseg;
        nseg = (c.nx + seg_len - 1) / seg_len;
        while (nseg > 1 && c.nx - (nseg - 1) * seg_len < 2 * M) {
            --nseg;
            seg_len = (c.nx + nseg - 1) / nseg;
            nseg = (c.nx + seg_len - 1) / seg_len;
        }
        *nseg_out = nseg;
        *len_out = seg_len;
    };
    split(tiles_run, &r.nseg, &r.seg_len);
    const int nseg = r.nseg;
    r.blocks = tiles_run * nseg;
    r.xcd_remap = (r.blocks % 8 == 0) ? 1 : 0;
    r.cap = cap;
    const size_t side_one = size_t(M) * size_t(lat) * size_t(c.ny) * size_t(c.nz) * elem_size(c.storage);
    r.side_bytes = size_t(nseg) * side_one;
    int nseg_max = nseg;
    if (r.nbands > 1 && last_segments) {
        // A round is bound by the latency of its plane iterations, not by its
        // bytes, so a short last band (FP64 512^3: 4 of 16 tile rows) takes
        // nearly the time of a full one; cut into more x segments it fills
        // the device and takes a fraction of it.
        const int last_rows = r.nty - (r.nbands - 1) * r.nty_band;
        int ns = 0, len = 0;
        split(last_rows * r.ntz, &ns, &len);
        if (ns > nseg) {
            r.nseg_last = ns;
            r.seg_len_last = len;
            r.side_off_last = align_up(r.side_bytes);
            r.side_bytes = r.side_off_last + size_t(ns) * side_one;
            nseg_max = ns;
        }
    }
    r.shell_bytes = r.nbands > 1 ? size_t(r.nbands) * 2u * size_t(M) * size_t(c.nz) * size_t(c.nx) * size_t(lat) *
                                       elem_size(c.storage)
                                 : 0;
    // D3Q19 in rounds keeps each band in step: a workgroup stores a plane
    // only once its neighbours have finished the previous iteration, so the
    // halo rows its tiles share are still in L2 (1024^3 FP32: 40.7 -> 37.4 ms
    // per pass; FP64 512^3 2 % faster, FP64 1024^3 unchanged).  One round
    // (512^3 FP32: 0.5 % slower with it) and D3Q15, with fewer bytes per plane
    // (1024^3: 6 % slower), run without the extra wait.  It only tightens the
    // wait of the hazard check; the slowest workgroup still never waits.
    r.lockstep = (r.nbands > 1 && lat == 19) ? 1 : 0;
    r.flag_stride = kFlagStride;
    r.flag_bytes = size_t(tiles * nseg_max + 1) * size_t(kFlagStride) * sizeof(int);
    *p = r;
    return LBM_OK;
}

// work buffer layout; plans use the device's co-residency cap
lbm_status layout(const lbm_config& c, int cap, MarchPlan plans[4], size_t off[6], size_t* total, std::string* why,
                  bool last_segments)
{
    const long long N = (long long)c.nx * c.ny * c.nz;
    size_t o = 0;
    off[0] = o;  // reduction partials
    o = align_up(o + size_t(SUM_BLOCKS) * 4 * sizeof(double));
    off[1] = o;  // final sums
    o = align_up(o + 4 * sizeof(double));
    off[2] = off[3] = off[4] = off[5] = 0;
    if (c.scheme == LBM_TWO_ARRAY) {
        off[2] = o;  // the second lattice of the plain scheme
        o = align_up(o + size_t(lat_of(c)) * size_t(N) * elem_size(c.storage));
    } else {
        size_t flags = 0, side = 0, shell = 0;
        // the merged schemes also run the shorter passes of a remainder of steps
        for (int M = 1; M <= 3; ++M) {
            if (M == 2 && c.scheme != LBM_SWAP2 && c.scheme != LBM_SWAP3) continue;
            if (M == 3 && c.scheme != LBM_SWAP3) continue;
            lbm_status st = make_plan(c, M, cap, &plans[M], why, last_segments);
            if (st != LBM_OK) return st;
            if (plans[M].flag_bytes > flags) flags = plans[M].flag_bytes;
            if (plans[M].side_bytes > side) side = plans[M].side_bytes;
            if (plans[M].shell_bytes > shell) shell = plans[M].shell_bytes;
        }
        off[3] = o;
        o = align_up(o + flags);
        off[4] = o;
        o = align_up(o + side);
        off[5] = o;
        o = align_up(o + shell);
    }
    *total = o;
    return LBM_OK;
}

int device_cap(const lbm_config& c, const MarchPlan& p)
{
    const bool walls = c.face[0] != LBM_PERIODIC || c.face[2] != LBM_PERIODIC || c.face[4] != LBM_PERIODIC;
    const bool force = c.use_force != 0;
    if (lat_of(c) != 19) return max_blocks_set(lat_of(c), c.storage, walls, force, p);
    switch (c.storage) {
    case LBM_F64: return max_blocks_f64(walls, force, p);
    case LBM_F32: return max_blocks_f32(walls, force, p);
    case LBM_F16_OFS: return max_blocks_f16(walls, force, p);
    default: return max_blocks_bf16(walls, force, p);
    }
}

hipError_t launch_march_pass(const lbm_config& cfg, const Geom& g, const MarchPlan& p, const PassBuffers& b,
                             bool force_timeout, hipStream_t s)
{
    MarchArgs a{};
    a.g = g;
    const bool inplace = b.src == b.dst;
    a.f = const_cast<void*>(b.src);
    a.fo = b.dst;
    a.inplace = inplace ? 1 : 0;
    a.side = b.side;
    a.force = b.force;
    a.flags = b.flags;
    a.nty = p.nty;
    a.ntz = p.ntz;
    a.nseg = p.nseg;
    a.seg_len = p.seg_len;
    a.ry = p.ry;
    a.rz = p.rz;
    a.xcd_remap = p.xcd_remap;
    a.fstride = p.flag_stride;
    a.spin_limit = force_timeout ? 4 : (1 << 22);
    a.need_bias = force_timeout ? (1 << 29) : p.lockstep;
    const bool walls = g.wall[0] || g.wall[1] || g.wall[2];
    const bool force = b.force != nullptr;
    // one (band, first/last rows) slab of the band boundary copy: [x][q][row][z]
    const size_t part = size_t(g.nx) * size_t(g.lat) * size_t(p.M) * size_t(g.nz) * elem_size(cfg.storage);
    const bool py = cfg.face[2] == LBM_PERIODIC;
    hipError_t e = hipSuccess;
    for (int band = 0; band < p.nbands && e == hipSuccess; ++band) {
        // one round: a band of tile rows; with one band, the whole plane
        MarchPlan pb = p;
        a.band_ty0 = band * p.nty_band;
        a.nty_band = std::min(p.nty_band, p.nty - a.band_ty0);
        if (band == p.nbands - 1 && p.nseg_last > 0) {
            // the short last band: its own x segments and their side planes
            a.nseg = p.nseg_last;
            a.seg_len = p.seg_len_last;
            a.side = b.side ? static_cast<unsigned char*>(b.side) + p.side_off_last : nullptr;
        }
        a.shell_lo = (inplace && band > 0) ? b.shell + (size_t(2 * (band - 1) + 1)) * part : nullptr;
        a.shell_hi = (inplace && p.nbands > 1 && band == p.nbands - 1 && py) ? b.shell : nullptr;
        // work items of the round; the grid is padded with idle workgroups to
        // a multiple of 8 (when they still fit) so that the XCD remap applies
        a.items = a.nty_band * p.ntz * a.nseg;
        // with the x axis cut into segments, non-temporal in-place stores
        // measured faster (256^3: +7 % periodic, +11 % with walls and a
        // force); with one segment, slower (512^3: -3 %)
        a.nt_store = a.nseg > 1 ? 1 : 0;
        const int padded = (a.items + 7) / 8 * 8;
        pb.blocks = padded <= p.cap ? padded : a.items;
        pb.xcd_remap = (pb.blocks % 8 == 0) ? 1 : 0;
        a.xcd_remap = pb.xcd_remap;
        if (g.lat != 19) {
            e = launch_march_set(g.lat, cfg.storage, walls, force, pb, a, s);
            continue;
        }
        switch (cfg.storage) {
        case LBM_F64: e = launch_march_f64(walls, force, pb, a, s); break;
        case LBM_F32: e = launch_march_f32(walls, force, pb, a, s); break;
        case LBM_F16_OFS: e = launch_march_f16(walls, force, pb, a, s); break;
        default: e = launch_march_bf16(walls, force, pb, a, s); break;
        }
    }
    return e;
}

}  // namespace lbm
