// Planner: label classification into the bundles I, J, P (Sec. 4), the
// dimension reordering heuristic (Sec. 7.3) with two GPU amendments (the P
// order follows the operand with its unit stride in P; an operand's
// unit-stride index goes to the front of its free bundle), scatter vectors
// (Sec. 6.1) and block strides (Sec. 6.2) at the tile granularity of the GPU
// kernel.
#include "plan.hpp"

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <sstream>

#include "tc.h"

namespace tc {

static thread_local std::string g_err;
void set_error(const std::string& msg) { g_err = msg; }
const char* last_error() { return g_err.c_str(); }

static int fail(int st, const std::string& msg) {
    set_error(msg);
    return st;
}

static int find(const TensorDesc& t, char l) {
    for (int i = 0; i < t.ndim; ++i)
        if (t.idx[i] == l) return i;
    return -1;
}

static std::string lab(char c) { return std::string(1, c); }

// Element span of a tensor (largest offset + 1), 0 when empty.
static int64_t span_of(const TensorDesc& t) {
    int64_t s = 1;
    for (int i = 0; i < t.ndim; ++i) {
        if (t.lens[i] == 0) return 0;
        s += (t.lens[i] - 1) * t.strides[i];
    }
    return s;
}

static int check_tensor(const TensorDesc& t, const char* name) {
    for (int i = 0; i < t.ndim; ++i) {
        if (t.lens[i] < 0) return fail(TC_ERR_EXTENT, std::string(name) + ": negative length");
        if (t.lens[i] > 1 && t.strides[i] <= 0)
            return fail(TC_ERR_STRIDE, std::string(name) + ": stride <= 0 on a dimension of length > 1");
        for (int j = i + 1; j < t.ndim; ++j)
            if (t.idx[i] == t.idx[j])
                return fail(TC_ERR_LABEL, std::string(name) + ": label '" + lab(t.idx[i]) + "' repeated");
    }
    return TC_OK;
}

// Sufficient check that distinct indices of C address distinct elements.
static int check_no_self_overlap(const TensorDesc& t) {
    std::vector<std::pair<int64_t, int64_t>> d;  // (stride, len)
    for (int i = 0; i < t.ndim; ++i) {
        if (t.lens[i] == 0) return TC_OK;  // empty tensor
        if (t.lens[i] > 1) d.push_back({t.strides[i], t.lens[i]});
    }
    std::sort(d.begin(), d.end());
    for (size_t i = 1; i < d.size(); ++i)
        if (d[i].first < d[i - 1].first * d[i - 1].second)
            return fail(TC_ERR_ALIAS, "C: dimensions overlap in memory (stride smaller than the previous extent)");
    return TC_OK;
}

void scatter_vector(const std::vector<Dim>& dims, int which, std::vector<int64_t>* out) {
    // which: 0 = X strides, 1 = Y strides, 2 = C strides
    int64_t total = 1;
    for (const Dim& d : dims) total *= d.len;
    out->assign((size_t)total, 0);
    if (total == 0) return;
    // colexicographic walk (first index fastest), offsets accumulated
    std::vector<int64_t> ctr(dims.size(), 0);
    int64_t off = 0;
    for (int64_t x = 0; x < total; ++x) {
        (*out)[(size_t)x] = off;
        for (size_t i = 0; i < dims.size(); ++i) {
            int64_t s = which == 0 ? dims[i].sX : which == 1 ? dims[i].sY : dims[i].sC;
            if (++ctr[i] < dims[i].len) {
                off += s;
                break;
            }
            off -= s * (dims[i].len - 1);
            ctr[i] = 0;
        }
    }
}

void scatter_vector_sub(const std::vector<Dim>& dims, int which, int a, int b, int64_t bx, int64_t by,
                        std::vector<int64_t>* out) {
    int64_t total = 1;
    for (const Dim& d : dims) total *= d.len;
    out->assign((size_t)total, 0);
    if (total == 0) return;
    auto st = [which](const Dim& d) { return which == 0 ? d.sX : which == 1 ? d.sY : d.sC; };
    const int64_t La = dims[(size_t)a].len, Lb = dims[(size_t)b].len, plane = La * Lb;
    for (int64_t x = 0; x < total; ++x) {
        // position inside the (a, b) plane: bands of `by` values of b, each
        // cut into blocks of `bx` values of a (the last band and block of a
        // ragged extent are shorter), a fastest inside a block
        const int64_t r = x % plane;
        int64_t rest = x / plane;
        const int64_t band = r / (La * by), r2 = r - band * La * by;
        const int64_t h = std::min(by, Lb - band * by);
        const int64_t blk = r2 / (bx * h), r3 = r2 - blk * bx * h;
        const int64_t w = std::min(bx, La - blk * bx);
        int64_t off = (blk * bx + r3 % w) * st(dims[(size_t)a]) + (band * by + r3 / w) * st(dims[(size_t)b]);
        for (size_t d = 0; d < dims.size(); ++d) {
            if ((int)d == a || (int)d == b) continue;
            off += (rest % dims[d].len) * st(dims[d]);
            rest /= dims[d].len;
        }
        (*out)[(size_t)x] = off;
    }
}

void block_strides(const int64_t* scat, int64_t len, int64_t b, int64_t* out) {
    int64_t nb = (len + b - 1) / b;
    for (int64_t i = 0; i < nb; ++i) {
        int64_t lo = i * b, hi = std::min(len, (i + 1) * b);
        if (hi - lo <= 1) {
            out[i] = 1;  // one entry: any stride describes it
            continue;
        }
        int64_t s = scat[lo + 1] - scat[lo];
        bool ok = s > 0;
        for (int64_t j = lo + 2; ok && j < hi; ++j) ok = (scat[j] - scat[j - 1] == s);
        out[i] = ok ? s : 0;
    }
}

static void sort_by(std::vector<Dim>* v, int which) {
    std::stable_sort(v->begin(), v->end(), [which](const Dim& a, const Dim& b) {
        int64_t sa = which == 0 ? a.sX : which == 1 ? a.sY : a.sC;
        int64_t sb = which == 0 ? b.sX : which == 1 ? b.sY : b.sC;
        return sa < sb;
    });
}

// Fold adjacent dims (x, y) when y's stride equals x's stride times x's
// length in every tensor that holds them (Sec. 7.3, step 2).  Folding keeps
// every scatter-vector entry unchanged; it shortens the index arithmetic.
static int fold(std::vector<Dim>* v, bool inX, bool inY, bool inC) {
    int folds = 0;
    bool changed = true;
    while (changed) {
        changed = false;
        for (size_t i = 0; i + 1 < v->size(); ++i) {
            Dim& x = (*v)[i];
            Dim& y = (*v)[i + 1];
            bool ok = (!inX || y.sX == x.sX * x.len) && (!inY || y.sY == x.sY * x.len) &&
                      (!inC || y.sC == x.sC * x.len);
            if (ok) {
                x.len *= y.len;
                x.labels += y.labels;
                v->erase(v->begin() + (long)i + 1);
                ++folds;
                changed = true;
                break;
            }
        }
    }
    return folds;
}

Plan::~Plan() {}

static int64_t prod(const std::vector<Dim>& v) {
    int64_t p = 1;
    for (const Dim& d : v) p *= d.len;
    return p;
}

int build_plan(const TensorDesc& A, const TensorDesc& B, const TensorDesc& C, int dtype, int mode,
               std::unique_ptr<Plan>* out) {
    if (!((dtype == TC_F64 && mode == TC_NATIVE) || (dtype == TC_F32 && (mode == TC_NATIVE || mode == TC_SPLIT_BF16X3))))
        return fail(TC_ERR_DTYPE, "unsupported dtype/mode combination");
    int st;
    if ((st = check_tensor(A, "A")) || (st = check_tensor(B, "B")) || (st = check_tensor(C, "C"))) return st;

    auto p = std::make_unique<Plan>();
    p->dtype = dtype;
    p->mode = mode;
    p->dA = A;
    p->dB = B;
    p->dC = C;

    // --- classify labels (Sec. 4): I = A&C, J = B&C, P = A&B -------------
    std::vector<Dim> I, J, P;
    for (int c = 0; c < C.ndim; ++c) {
        char l = C.idx[c];
        int a = find(A, l), b = find(B, l);
        if ((a >= 0) == (b >= 0))
            return fail(TC_ERR_LABEL, "label '" + lab(l) + "' of C must appear in exactly one of A, B");
        int64_t len2 = a >= 0 ? A.lens[a] : B.lens[b];
        if (len2 != C.lens[c]) return fail(TC_ERR_EXTENT, "label '" + lab(l) + "' has different lengths");
        Dim d;
        d.len = C.lens[c];
        d.sC = C.strides[c];
        d.labels = lab(l);
        if (a >= 0) {
            d.sX = A.strides[a];
            I.push_back(d);
        } else {
            d.sY = B.strides[b];
            J.push_back(d);
        }
    }
    for (int a = 0; a < A.ndim; ++a) {
        char l = A.idx[a];
        if (find(C, l) >= 0) continue;
        int b = find(B, l);
        if (b < 0) return fail(TC_ERR_LABEL, "label '" + lab(l) + "' appears only in A");
        if (B.lens[b] != A.lens[a]) return fail(TC_ERR_EXTENT, "label '" + lab(l) + "' has different lengths");
        Dim d;
        d.len = A.lens[a];
        d.sX = A.strides[a];
        d.sY = B.strides[b];
        d.labels = lab(l);
        P.push_back(d);
    }
    for (int b = 0; b < B.ndim; ++b)
        if (find(A, B.idx[b]) < 0 && find(C, B.idx[b]) < 0)
            return fail(TC_ERR_LABEL, "label '" + lab(B.idx[b]) + "' appears only in B");
    if ((st = check_no_self_overlap(C))) return st;

    p->spanA = span_of(A);
    p->spanB = span_of(B);
    p->spanC = span_of(C);

    // --- empty extents --------------------------------------------------
    for (const Dim& d : I) p->noop |= d.len == 0;
    for (const Dim& d : J) p->noop |= d.len == 0;
    for (const Dim& d : P) p->k_empty |= d.len == 0;

    // --- reordering heuristic (Sec. 7.3) ---------------------------------
    // 1. drop length-1 dims
    auto drop1 = [&](std::vector<Dim>* v) {
        size_t before = v->size();
        v->erase(std::remove_if(v->begin(), v->end(), [](const Dim& d) { return d.len == 1; }), v->end());
        p->dropped += (int)(before - v->size());
    };
    drop1(&I);
    drop1(&J);
    drop1(&P);
    // 3. sort I and J by increasing stride in C
    sort_by(&I, 2);
    sort_by(&J, 2);
    // 4. C^T = B^T A^T when C's unit stride lies in J
    if (!J.empty() && J[0].sC == 1) {
        p->swapped = true;
        std::swap(I, J);
        for (Dim& d : I) std::swap(d.sX, d.sY);
        for (Dim& d : J) std::swap(d.sX, d.sY);
        for (Dim& d : P) std::swap(d.sX, d.sY);
    }
    // 5. order P by increasing stride in A (X after the swap), as printed
    sort_by(&P, 0);
    auto names = [](const std::vector<Dim>& v) {
        std::string out;
        for (const Dim& d : v) out += d.labels;
        return out;
    };
    p->paper_order = names(I) + "|" + names(J) + "|" + names(P);
    // GPU amendment 1.  Each operand is gathered with its lanes along its
    // unit-stride index, so P is sorted by the stride of whichever operand
    // has its unit stride inside P (ties: X).
    bool ux = false, uy = false;
    for (const Dim& d : P) {
        ux |= d.sX == 1;
        uy |= d.sY == 1;
    }
    if (!ux && uy) sort_by(&P, 1);
    // GPU amendment 2.  The C-stride sort of step 3 can leave an operand's
    // unit-stride index behind another index of its free bundle (C and the
    // operand order the bundle's indices differently, Sec. 7.3 and Sec. 9.3);
    // then neither the m (n) nor the k direction of that operand is unit
    // stride and every lane of its gather reads a separate line.  The gathers
    // are repeated for every tile column (row) while C is written once, and
    // the tile stores' lanes run along n in most fragment layouts, so the
    // operand's unit-stride index is moved to the front of its free bundle.
    auto unit_first = [](std::vector<Dim>* v, int which) {
        for (size_t i = 1; i < v->size(); ++i) {
            const int64_t s = which == 0 ? (*v)[i].sX : (*v)[i].sY;
            if (s == 1) {
                Dim d = (*v)[i];
                v->erase(v->begin() + (long)i);
                v->insert(v->begin(), d);
                return 1;
            }
        }
        return 0;
    };
    if (!(!I.empty() && I[0].sX == 1) && !(!P.empty() && P[0].sX == 1)) p->unit_moves += unit_first(&I, 0);
    if (!(!J.empty() && J[0].sY == 1) && !(!P.empty() && P[0].sY == 1)) p->unit_moves += unit_first(&J, 1);
    // 2. fold dimensions contiguous in every tensor holding them (after the
    //    sort, so adjacency refers to the planned order)
    p->folds += fold(&I, true, false, true);
    p->folds += fold(&J, false, true, true);
    p->folds += fold(&P, true, true, false);

    // GPU amendment 3.  When X and Y have their unit strides on two
    // different P dims (the storage orders of A and B disagree inside the
    // contracted bundle, Sec. 7.3 and Sec. 9.2-9.3), any P order leaves one
    // operand strided along k, and a k stage of it touches one line per
    // element.  The k order is then sub-blocked instead (the paper's
    // sub-division of dimensions, applied to the k loop): a stage of KT
    // entries covers bx values of X's unit-stride dim times by values of
    // Y's, so both operands read runs of contiguous elements.  Any order of
    // the k sum gives the same contraction.  Sub-blocks shorten X's runs
    // along k, so they are used only when Y's best plain gather (lanes along
    // J[0] or P[0]) has a stride longer than the run the sub-blocks give Y.
    {
        int ua = -1, ub = -1;
        for (size_t i = 0; i < P.size(); ++i) {
            if (P[i].sX == 1 && ua < 0) ua = (int)i;
            if (P[i].sY == 1 && ub < 0) ub = (int)i;
        }
        const int64_t KT = tile_table(dtype, mode)[0].KT;
        const int64_t bx = ua >= 0 ? std::min<int64_t>(KT == 16 ? 4 : 8, P[(size_t)ua].len) : 1;
        const int64_t by = ub >= 0 ? std::max<int64_t>(1, std::min<int64_t>(KT / bx, P[(size_t)ub].len)) : 1;
        int64_t ybest = P.empty() ? 0 : P[0].sY;
        if (!J.empty() && (ybest == 0 || J[0].sY < ybest)) ybest = J[0].sY;
        if (ua >= 0 && ub >= 0 && ua != ub && ybest > by) {
            p->sub_a = ua;
            p->sub_b = ub;
            p->sub_bx = bx;
            p->sub_by = by;
        }
    }

    p->I = I;
    p->J = J;
    p->P = P;
    p->m = prod(I);
    p->n = prod(J);
    p->k = prod(P);
    if (p->noop) p->m = p->n = 0;

    // --- offsets width ------------------------------------------------------
    // 32-bit offsets need element spans below 2^31; the 32-bit kernels also
    // address A and B with bounds-checked buffer loads whose byte offsets
    // must stay below 2^31.
    const int64_t lim = (int64_t)0x7fffffff;
    const int64_t elt = dtype == TC_F64 ? 8 : 4;
    p->off64 = p->spanA * elt > lim || p->spanB * elt > lim || p->spanC > lim || p->m > lim || p->n > lim ||
               p->k > lim;

    // --- scatter vectors (Sec. 6.1) --------------------------------------
    if (!p->noop) {
        scatter_vector(I, 0, &p->rX);
        scatter_vector(I, 2, &p->rC);
        scatter_vector(J, 1, &p->cY);
        scatter_vector(J, 2, &p->cC);
        if (!p->k_empty && p->sub_a >= 0) {
            scatter_vector_sub(P, 0, p->sub_a, p->sub_b, p->sub_bx, p->sub_by, &p->cX);
            scatter_vector_sub(P, 1, p->sub_a, p->sub_b, p->sub_bx, p->sub_by, &p->rY);
        } else if (!p->k_empty) {
            scatter_vector(P, 0, &p->cX);
            scatter_vector(P, 1, &p->rY);
        }
    }
    // --- lane-fast dimension of each operand for the gather --------------
    if (!I.empty() && I[0].sX == 1) p->x_lanes_m = true;
    else if (!P.empty() && P[0].sX == 1) p->x_lanes_m = false;
    else if (!I.empty() && !P.empty()) p->x_lanes_m = I[0].sX <= P[0].sX;
    else p->x_lanes_m = !I.empty();
    if (!J.empty() && J[0].sY == 1) p->y_lanes_n = true;
    else if (!P.empty() && P[0].sY == 1) p->y_lanes_n = false;
    else if (p->sub_a >= 0) p->y_lanes_n = false;  // runs of Y along its unit-stride P dim
    else if (!J.empty() && !P.empty()) p->y_lanes_n = J[0].sY <= P[0].sY;
    else p->y_lanes_n = !J.empty();

    p->tile = choose_tile(*p);
    set_plan_tile(p.get(), p->tile);
    *out = std::move(p);
    return TC_OK;
}

void set_plan_tile(Plan* p, int tile) {
    const TileCfg& t = tile_table(p->dtype, p->mode)[tile];
    p->tile = tile;
    auto bs = [](const std::vector<int64_t>& v, int64_t b, std::vector<int64_t>* out) {
        out->assign((size_t)((int64_t)v.size() + b - 1) / b, 0);
        if (!v.empty()) block_strides(v.data(), (int64_t)v.size(), b, out->data());
    };
    bs(p->cX, t.KT, &p->kbsX);
    bs(p->rY, t.KT, &p->kbsY);
    bs(p->rX, t.MT, &p->rbsX);
    bs(p->cY, t.NT, &p->cbsY);
    bs(p->rC, t.MT, &p->rbsC);
    bs(p->cC, t.NT, &p->cbsC);
    p->tiles_m = (p->m + t.MT - 1) / t.MT;
    p->tiles_n = (p->n + t.NT - 1) / t.NT;
    int64_t rv = 0, cv = 0;
    for (int64_t v : p->rbsC) rv += v != 0;
    for (int64_t v : p->cbsC) cv += v != 0;
    p->c_tiles_regular = rv * cv;
    p->k_blocks_regular_x = 0;
    p->k_blocks_regular_y = 0;
    for (int64_t v : p->kbsX) p->k_blocks_regular_x += v != 0;
    for (int64_t v : p->kbsY) p->k_blocks_regular_y += v != 0;
    for (auto& d : p->dev) d.bytes = 0;  // device copies are stale (freed lazily)
}

// Cost model over the compiled tiles: the per-CU compute time of the tile
// rounds (wave quantisation over the chip's 256 CUs, with up to `occ`
// workgroups resident per CU and the measured rate for that residency),
// bounded below by the time to stream every tile's A and B slivers from the
// caches (small tiles re-read the operands many times), plus the C update of
// each round at the tile's relative store speed (what decides short-k,
// output-bound shapes).  For a problem of a batch the rounds are fractional
// (the other problems fill the chip).  Among tiles bound by the stream term
// the faster computing one wins; earlier tiles win exact ties.
int choose_tile(const Plan& p, bool batched) {
    const TileCfg* tab = tile_table(p.dtype, p.mode);
    const TileRate* rate = rate_table(p.dtype, p.mode);
    const int nt = tile_count(p.dtype, p.mode);
    // operands stream from the caches at about 8 TB/s in a single
    // contraction; in a batch the caches hold many problems' panels at once,
    // and 4 TB/s fits the batches measured
    const double cus = 256.0, cache_bw = batched ? 4e12 : 8e12, hbm_bw = 5e12;
    const double esize = p.dtype == TC_F64 ? 8.0 : 4.0;
    const double k = (double)std::max<int64_t>(p.k, 1);
    int best = 0;
    double best_t = 1e300;
    for (int i = 0; i < nt; ++i) {
        const TileCfg& t = tab[i];
        // batches run every problem's class from one persistent kernel that
        // holds all four lane variants of the tile; for the pinwheels that
        // kernel spills registers, so by default batches use the other layouts
        if (batched && (t.layout == 1 || t.layout == 2 || t.layout == 4)) continue;
        if (t.layout == 4 && split_pack_bytes(t, p.m, p.n, p.k) > kMaxSplitPanelBytes) continue;
        // the 32 x 32 tiles win single small launches by parallelism, which a
        // batch supplies from its other problems; inside batches they ran
        // slower than the larger tiles
        if (batched && t.MT * t.NT <= 32 * 32) continue;
        const double tiles = (double)((p.m + t.MT - 1) / t.MT) * (double)((p.n + t.NT - 1) / t.NT);
        // a batch keeps every CU at the tile's full residency with the tiles
        // of all its problems, so a problem's share is its padded work at that
        // rate, with no rounding to waves of the chip
        const double w = batched ? (double)rate[i].occ : std::min((double)rate[i].occ, std::ceil(tiles / cus));
        const double rounds = batched ? tiles / (cus * w) : std::ceil(tiles / (cus * w));
        const double r = (w >= 2.0 ? rate[i].r2 : rate[i].r1) * 1e12 / cus;  // flop/s of one CU
        const double compute = rounds * w * 2.0 * t.MT * t.NT * k / r;
        const double stream = tiles * (double)(t.MT + t.NT) * k * esize / cache_bw;
        const double store = rounds * w * cus * (double)t.MT * t.NT * esize / (hbm_bw * rate[i].store);
        // where the streaming bound decides, the tile that computes faster
        // wins the tie
        // the packed split tile adds its split-and-pack pass: each operand
        // element gathered once (4 bytes) and written once as hi and lo
        // (4 bytes), at about 5 TB/s, plus a second launch
        const double pack = t.layout == 4 ? (double)split_pack_bytes(t, p.m, p.n, p.k) * 2.0 / 5e12 + 3e-6 : 0.0;
        const double time = std::max(compute, stream) + store + pack + 0.01 * compute;
        if (time < best_t * 0.999) {
            best_t = time;
            best = i;
        }
    }
    return best;
}

std::string plan_signature(const Plan& p) {
    std::ostringstream os;
    os << p.dtype << '/' << p.mode << '/' << (p.swapped ? 1 : 0);
    auto dims = [&](const std::vector<Dim>& v) {
        os << '[';
        for (const Dim& d : v) os << d.len << ':' << d.sX << ',' << d.sY << ',' << d.sC << ';';
        os << ']';
    };
    dims(p.I);
    dims(p.J);
    dims(p.P);
    return os.str();
}

static void json_vec(std::ostringstream& os, const char* name, const std::vector<int64_t>& v, bool last = false) {
    os << '"' << name << "\":[";
    for (size_t i = 0; i < v.size(); ++i) os << (i ? "," : "") << v[i];
    os << ']' << (last ? "" : ",");
}

static void json_dims(std::ostringstream& os, const char* name, const std::vector<Dim>& v) {
    os << '"' << name << "\":[";
    for (size_t i = 0; i < v.size(); ++i)
        os << (i ? "," : "") << "{\"labels\":\"" << v[i].labels << "\",\"len\":" << v[i].len << ",\"sX\":" << v[i].sX
           << ",\"sY\":" << v[i].sY << ",\"sC\":" << v[i].sC << '}';
    os << "],";
}

std::string describe_plan(const Plan& p) {
    const TileCfg& t = tile_table(p.dtype, p.mode)[p.tile];
    std::ostringstream os;
    os << '{';
    os << "\"dtype\":" << p.dtype << ",\"mode\":" << p.mode << ",\"swapped\":" << (p.swapped ? "true" : "false")
       << ",\"m\":" << p.m << ",\"n\":" << p.n << ",\"k\":" << p.k << ",\"noop\":" << (p.noop ? "true" : "false")
       << ",\"k_empty\":" << (p.k_empty ? "true" : "false") << ",\"off64\":" << (p.off64 ? "true" : "false")
       << ",\"folds\":" << p.folds << ",\"dropped\":" << p.dropped << ",\"unit_moves\":" << p.unit_moves
       << ",\"paper_order\":\"" << p.paper_order << "\",";
    if (p.sub_a >= 0)
        os << "\"k_sub\":{\"a\":" << p.sub_a << ",\"b\":" << p.sub_b << ",\"bx\":" << p.sub_bx << ",\"by\":" << p.sub_by
           << "},";
    else
        os << "\"k_sub\":null,";
    json_dims(os, "I", p.I);
    json_dims(os, "J", p.J);
    json_dims(os, "P", p.P);
    os << "\"x_lanes\":\"" << (p.x_lanes_m ? "m" : "k") << "\",\"y_lanes\":\"" << (p.y_lanes_n ? "n" : "k") << "\",";
    os << "\"tile\":" << p.tile << ",\"MT\":" << t.MT << ",\"NT\":" << t.NT << ",\"KT\":" << t.KT
       << ",\"waves\":" << t.waves() << ",\"tiles_m\":" << p.tiles_m << ",\"tiles_n\":" << p.tiles_n
       << ",\"c_tiles_regular\":" << p.c_tiles_regular << ",\"k_blocks\":" << p.kbsX.size()
       << ",\"k_blocks_regular_x\":" << p.k_blocks_regular_x << ",\"k_blocks_regular_y\":" << p.k_blocks_regular_y
       << ",\"layout\":" << t.layout << ",\"workspace_bytes\":"
       << (t.layout == 4 && !p.k_empty ? split_pack_bytes(t, p.m, p.n, p.k) : 0) << ',';
    bool small = (int64_t)std::max({p.rX.size(), p.cY.size(), p.cX.size()}) <= TC_DESCRIBE_MAX_VECTOR;
    if (small) {
        json_vec(os, "rscat_X", p.rX);
        json_vec(os, "cscat_X", p.cX);
        json_vec(os, "rscat_Y", p.rY);
        json_vec(os, "cscat_Y", p.cY);
        json_vec(os, "rscat_C", p.rC);
        json_vec(os, "cscat_C", p.cC);
        json_vec(os, "kbs_X", p.kbsX);
        json_vec(os, "kbs_Y", p.kbsY);
        json_vec(os, "rbs_X", p.rbsX);
        json_vec(os, "cbs_Y", p.cbsY);
        json_vec(os, "rbs_C", p.rbsC);
        json_vec(os, "cbs_C", p.cbsC);
    }
    os << "\"vectors\":" << (small ? "true" : "false") << '}';
    return os.str();
}

}  // namespace tc
