// Planner: access-region inference and distributions.
//
// Region inference (Sec. 2.3, Sec. 2.4).  For a superblock (a box of whole
// thread blocks) and one annotated access, the region is the dense bounding
// box of every element the superblock's threads touch, clipped to the
// array's domain.  Global indices are rewritten as g = B*b + l (block index b,
// index l inside the block); b and l then range independently over a box, so
// the minimum and maximum of each affine bound sit at corners of that box and
// are computed exactly, without enumerating threads.
//
// Distributions (Sec. 2.2): a BLOCK policy cuts every axis into pieces of a
// fixed length (row-wise, column-wise, tiled); CUSTOM takes explicit disjoint
// boxes that cover the domain; STENCIL stores each BLOCK core with a halo of
// replicas of its neighbours' elements.
#include <algorithm>

#include "lt_internal.h"

namespace lt {

void var_ranges(int nd, const int64_t *blk_lo, const int64_t *blk_hi,
                const int64_t *block, VarRange *r) {
    for (int k = 0; k < NVAR; ++k) r->lo[k] = r->hi[k] = 0;
    for (int a = 0; a < nd; ++a) {
        r->lo[3 + a] = blk_lo[a];
        r->hi[3 + a] = blk_hi[a] - 1;  // block index
        r->lo[6 + a] = 0;
        r->hi[6 + a] = block[a] - 1;   // index inside the block
    }
}

// Substitutes g_a = B_a * b_a + l_a and evaluates scalar parameters.
static void normalize(const Affine &f, int nd, const int64_t *block,
                      const int64_t *params, int64_t *c0, int64_t *coef) {
    *c0 = f.c0;
    for (int q = 0; q < MAXPARAM; ++q) *c0 += f.p[q] * params[q];
    for (int k = 0; k < NVAR; ++k) coef[k] = 0;
    for (int a = 0; a < 3; ++a) {
        int64_t g = f.v[a];
        int64_t B = a < nd ? block[a] : 1;
        coef[3 + a] += f.v[3 + a] + g * B;
        coef[6 + a] += f.v[6 + a] + g;
    }
}

static int64_t form_min(int64_t c0, const int64_t *coef, const VarRange &vr) {
    int64_t s = c0;
    for (int k = 3; k < NVAR; ++k) s += coef[k] >= 0 ? coef[k] * vr.lo[k] : coef[k] * vr.hi[k];
    return s;
}

static int64_t form_max(int64_t c0, const int64_t *coef, const VarRange &vr) {
    int64_t s = c0;
    for (int k = 3; k < NVAR; ++k) s += coef[k] >= 0 ? coef[k] * vr.hi[k] : coef[k] * vr.lo[k];
    return s;
}

bool access_region(const Access &a, int nd_grid, const int64_t *block,
                   const VarRange &vr, const int64_t *params, const Array *arr,
                   Box *out) {
    *out = Box();
    for (int x = 0; x < arr->ndim; ++x) {
        const IndexSpec &ix = a.idx[x];
        int64_t lc0 = 0, hc0 = arr->shape[x] - 1;
        int64_t lco[NVAR] = {0}, hco[NVAR] = {0};
        if (ix.has_lo) normalize(ix.lo, nd_grid, block, params, &lc0, lco);
        if (ix.has_hi) normalize(ix.hi, nd_grid, block, params, &hc0, hco);
        // a slice whose width hi - lo is a negative constant is empty for
        // every thread; a width that varies is bounded conservatively
        bool width_const = true;
        for (int k = 0; k < NVAR; ++k)
            if (hco[k] != lco[k]) width_const = false;
        if (width_const && hc0 < lc0) return false;
        int64_t lo = form_min(lc0, lco, vr);
        int64_t hi = form_max(hc0, hco, vr);
        lo = std::max<int64_t>(lo, 0);
        hi = std::min<int64_t>(hi, arr->shape[x] - 1);
        if (lo > hi) return false;
        out->lo[x] = lo;
        out->hi[x] = hi + 1;
    }
    return true;
}

lt_status make_chunks(Ctx *ctx, Array *arr, const lt_dist *dist) {
    const int nd = arr->ndim;
    std::vector<Box> boxes;
    if (!dist || dist->kind == LT_DIST_BLOCK || dist->kind == LT_DIST_STENCIL) {
        arr->dist_kind = LT_DIST_BLOCK;
        if (dist && dist->kind == LT_DIST_STENCIL) {
            for (int a = 0; a < MAXD; ++a) {
                int64_t h = a < nd ? dist->halo[a] : 0;
                if (h < 0) return set_err(ctx, LT_ERR_INVALID, "negative halo on axis %d", a);
                // along the contiguous axis the stored halo is a whole number
                // of 16-byte words, so rows of a chunk keep 16-byte alignment
                // (vector loads) whenever the core width allows it
                const int64_t w = arr->esz < 16 ? 16 / arr->esz : 1;
                if (a == nd - 1 && h > 0) h = (h + w - 1) / w * w;
                arr->halo[a] = h;
                if (h > 0) arr->has_halo = true;
            }
        }
        for (int a = 0; a < MAXD; ++a) {
            int64_t c = (dist && a < nd) ? dist->chunk[a] : 0;
            if (c < 0) return set_err(ctx, LT_ERR_INVALID, "negative chunk extent on axis %d", a);
            if (a >= nd) c = 1;
            else if (c == 0 || c > arr->shape[a]) c = arr->shape[a];
            arr->dist_chunk[a] = c;
            arr->nch[a] = a < nd ? (arr->shape[a] + c - 1) / c : 1;
        }
        int64_t total = arr->nch[0] * arr->nch[1] * arr->nch[2];
        if (total > (int64_t)1 << 24) return set_err(ctx, LT_ERR_INVALID, "too many chunks (%lld)", (long long)total);
        for (int64_t i = 0; i < arr->nch[0]; ++i)
            for (int64_t j = 0; j < arr->nch[1]; ++j)
                for (int64_t k = 0; k < arr->nch[2]; ++k) {
                    Box b;
                    int64_t idx[3] = {i, j, k};
                    for (int a = 0; a < nd; ++a) {
                        b.lo[a] = idx[a] * arr->dist_chunk[a];
                        b.hi[a] = std::min(arr->shape[a], b.lo[a] + arr->dist_chunk[a]);
                    }
                    boxes.push_back(b);
                }
        arr->row_slab = !arr->has_halo;  // overlapping chunks never form one dense slab
        for (int a = 1; a < nd; ++a)
            if (arr->nch[a] != 1) arr->row_slab = false;
    } else if (dist->kind == LT_DIST_CUSTOM) {
        arr->dist_kind = LT_DIST_CUSTOM;
        if (dist->nboxes <= 0 || !dist->boxes) return set_err(ctx, LT_ERR_INVALID, "custom distribution without boxes");
        Box dom;
        for (int a = 0; a < nd; ++a) dom.hi[a] = arr->shape[a];
        int64_t vol = 0;
        for (int i = 0; i < dist->nboxes; ++i) {
            Box b;
            for (int a = 0; a < nd; ++a) {
                b.lo[a] = dist->boxes[i].lo[a];
                b.hi[a] = dist->boxes[i].hi[a];
            }
            if (b.empty(nd) || !dom.contains(b, nd))
                return set_err(ctx, LT_ERR_INVALID, "custom chunk %d is empty or outside the domain", i);
            for (auto &o : boxes)
                if (!intersect(o, b, nd).empty(nd))
                    return set_err(ctx, LT_ERR_INVALID, "custom chunk %d overlaps another chunk", i);
            vol += b.volume(nd);
            boxes.push_back(b);
        }
        if (vol != dom.volume(nd)) return set_err(ctx, LT_ERR_INVALID, "custom chunks do not cover the domain");
        arr->row_slab = true;
        for (auto &b : boxes)
            for (int a = 1; a < nd; ++a)
                if (b.lo[a] != 0 || b.hi[a] != arr->shape[a]) arr->row_slab = false;
        if (arr->row_slab)
            std::sort(boxes.begin(), boxes.end(), [](const Box &x, const Box &y) { return x.lo[0] < y.lo[0]; });
    } else {
        return set_err(ctx, LT_ERR_INVALID, "unknown distribution kind %d", dist->kind);
    }
    for (size_t i = 0; i < boxes.size(); ++i) {
        Chunk *c = new Chunk();
        c->id = ctx->next_chunk_id++;
        c->arr = arr;
        c->index = (int)i;
        c->core = boxes[i];
        c->box = boxes[i];
        for (int a = 0; a < nd; ++a) {
            c->box.lo[a] = std::max<int64_t>(0, c->core.lo[a] - arr->halo[a]);
            c->box.hi[a] = std::min<int64_t>(arr->shape[a], c->core.hi[a] + arr->halo[a]);
        }
        c->elems = c->box.volume(nd);
        c->bytes = c->elems * arr->esz;
        // dense row-major storage of the chunk box on the device
        int64_t s = 1;
        for (int a = MAXD - 1; a >= 0; --a) {
            c->dev_stride[a] = s;
            s *= (a < nd) ? (c->box.hi[a] - c->box.lo[a]) : 1;
        }
        arr->chunks.push_back(c);
    }
    if (arr->has_halo) {
        // halo pieces: the parts of a chunk's stored box owned by other chunks
        for (Chunk *c : arr->chunks) {
            std::vector<Chunk *> owners;
            chunks_overlapping(arr, c->box, &owners);
            for (Chunk *k : owners) {
                if (k == c) continue;
                HaloSrc h;
                h.k = k;
                h.box = intersect(k->core, c->box, nd);
                if (!h.box.empty(nd)) c->halo.push_back(h);
            }
        }
    }
    return LT_OK;
}

Chunk *enclosing_chunk(const Array *arr, const Box &r) {
    const int nd = arr->ndim;
    std::vector<Chunk *> owners;
    chunks_overlapping(arr, r, &owners);
    // prefer the owner of the region's first element, then any owner
    for (Chunk *c : owners)
        if (c->core.contains_point(r.lo, nd) && c->box.contains(r, nd)) return c;
    for (Chunk *c : owners)
        if (c->box.contains(r, nd)) return c;
    return nullptr;
}

bool halo_stale(const Chunk *c, const Box &region) {
    const int nd = c->arr->ndim;
    for (const HaloSrc &h : c->halo)
        if ((!h.valid || h.ver < h.k->version) && !intersect(h.box, region, nd).empty(nd)) return true;
    return false;
}

void chunks_overlapping(const Array *arr, const Box &r, std::vector<Chunk *> *out) {
    out->clear();
    const int nd = arr->ndim;
    if (arr->dist_kind == LT_DIST_BLOCK) {
        int64_t lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
        for (int a = 0; a < 3; ++a) {
            if (a < nd) {
                lo[a] = r.lo[a] / arr->dist_chunk[a];
                hi[a] = (r.hi[a] - 1) / arr->dist_chunk[a];
            }
        }
        for (int64_t i = lo[0]; i <= hi[0]; ++i)
            for (int64_t j = lo[1]; j <= hi[1]; ++j)
                for (int64_t k = lo[2]; k <= hi[2]; ++k)
                    out->push_back(arr->chunks[(i * arr->nch[1] + j) * arr->nch[2] + k]);
    } else {
        for (Chunk *c : arr->chunks)
            if (!intersect(c->core, r, nd).empty(nd)) out->push_back(c);
    }
}

}  // namespace lt
