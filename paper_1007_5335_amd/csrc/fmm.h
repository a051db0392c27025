// fmm.h -- the FMM plan: a uniform-depth sparse quadtree over up to three
// point sets (charges, dipoles, target-only points), its interaction lists and
// the per-level translation operators of the modified-Helmholtz expansions.
//
// Expansions (alpha-scaled coordinates w = (y - c)/alpha, F^I_n(w) =
// I_n(|w|) e^{i n arg w}, F^K_n(w) = K_n(|w|) e^{i n arg w}):
//   multipole  phi(x) = sum_n M_n F^K_n((x - c)/alpha),
//              charge q at y:  M_n = q conj(F^I_n(w))          (Graf's addition theorem)
//              dipole D = d (n_x + i n_y):
//                   M_n = (1/(2 alpha)) [D conj(F^I_{n+1}(w)) + conj(D) conj(F^I_{n-1}(w))]
//   local      phi(x) = sum_m L_m F^I_m((x - c)/alpha)
//   M2L        L_m = (-1)^m sum_n M_n F^K_{n-m}((c_t - c_s)/alpha)
//   M2M, L2L   shifts by F^I_{n-k}(e), e = (child centre - parent centre)/alpha
// Coefficients are stored scaled per level, Mh_n = M_n / I_n(R_l) and
// Lh_m = L_m I_m(R_l), with R_l the box half-diagonal over alpha, so that every
// stored quantity and every operator entry is O(1) (no overflow in FP32).
// Only n = 0..p is stored (M_{-n} = conj(M_n) for real strengths) as the real
// vector [Re M_0, Re M_1, Im M_1, ..., Re M_p, Im M_p] of P = 2p + 1 entries,
// padded with zeros to Pp (a multiple of 16).
#pragma once

#include <map>

#include "sums.h"
#include "yk_internal.h"

namespace yk {

constexpr int kMaxLevel = 15;          // Morton keys carry 2 x 15 bits (+ 2 type bits)
constexpr int kNumV = 27;              // V-list slots per box (per parity class)
constexpr int kNumOff = 40;            // distinct V-list offsets in [-3,3]^2 minus [-1,1]^2

struct LevelInfo {
    int64_t begin = 0, end = 0;        // global box index range
    double side = 0;                   // box side
    double R = 0;                      // half-diagonal / alpha
};

// Boxes of one target mask that take part in the downward pass.
struct ActiveSet {
    DevBuf<int32_t> m2l_boxes;         // active boxes of levels lmin..L, sorted by (level, class)
    DevBuf<int4> m2l_tiles;            // {level, class, start, count} into m2l_boxes
    int n_tiles = 0;
    DevBuf<int4> m2l_tiles_w;          // the same boxes in tiles of up to 128 (FP32 M2L)
    int n_tiles_w = 0;
    // sparse M2L (trees whose V lists are mostly empty, such as a boundary
    // tree): the non-empty translations bucketed by (level, offset), tiles
    // {level, offset id, start, count} of up to 64 (target, source) pairs
    bool m2l_sparse = false;
    DevBuf<int4> m2l_ptiles;
    int n_ptiles = 0;
    DevBuf<int32_t> m2l_ptgt, m2l_psrc, m2l_piota;
    // partial rows of M2L launches whose workgroups share output rows (sparse
    // M2L; split slots on trees of few tiles), summed in a fixed order: for
    // the sparse form, per target box (csr_tgt) its translations
    // csr_rows[csr_off[t] .. csr_off[t+1]) in increasing index
    DevBuf<double> m2l_slab;
    DevBuf<int32_t> csr_tgt, csr_off, csr_rows;
    int64_t n_csr_tgt = 0, n_ptrans = 0;
    std::vector<int64_t> l2l_begin, l2l_count;   // per level: active boxes (children) list slices
    DevBuf<int32_t> l2l_boxes;         // active boxes of levels lmin+1..L (level-major)
    std::vector<int> tile_begin, tile_count;     // per level: slice of m2l_tiles
    DevBuf<int32_t> leaves;            // active leaves (leaf-local indices)
    int64_t n_leaves = 0;
    DevBuf<int2> leaf_items;           // {leaf, first target} work items of <= 64 targets
    std::vector<int64_t> item_lev_begin;   // adaptive tree: items by class 2 level + (a coarser
                                           // leaf touches it), 2 (L + 1) + 1 offsets
    int64_t n_items = 0;
    int64_t n_m2l_boxes = 0;
    // work counts (for measurement)
    int64_t pairs_q = 0, pairs_d = 0, m2l_trans = 0, l2p_points = 0;
    // cached near-field interactions (points and alpha only): per item, source
    // major and target minor, in the U-list order of the near kernel; charge
    // entries K0, dipole entries the pair (dx, dy) 4 K1(z)/z (scaled units)
    DevBuf<int64_t> item_qoff, item_doff;   // entry offsets per item
    int64_t near_q_len = 0, near_d_len = 0; // entries (dipole entries are pairs)
    int64_t near_q_vals = 0;                // charge entries other than alignment padding
    DevBuf<double> nq64, nd64;
    DevBuf<float> nq32, nd32;
    bool near64 = false, near32 = false;     // built
    // symmetric charge values (the charges among the targets, at most 64 per
    // leaf): each pair block of neighbouring leaves stored once, by the
    // leaf of smaller index, which also adds it, transposed, into the other
    // leaf's incoming slot.  Per item a descriptor and the slot each U-list
    // entry writes (-1: none); per leaf the first slot entry and the number
    // of slots.
    bool near_sym = false;
    DevBuf<int32_t> sym_desc;          // per item: U-list ranges and target ranges (52 entries)
    DevBuf<int64_t> sym_desc_dst;      // per item: the incoming slot of each U-list entry
    DevBuf<int64_t> inc_base;
    DevBuf<int32_t> inc_cnt;
    DevBuf<double> inc;
    int64_t inc_len = 0;
    // the cache's layout (offsets, symmetric slots, descriptors) is built on
    // the first evaluation that reads the cache (ensure_near_layout), from
    // these host copies
    bool layout = false;
    int mask = 0;
    std::vector<int2> h_items;
    std::vector<int64_t> h_sq, h_sd, h_tcnt;   // per leaf: neighbouring charges, dipoles; targets
    std::vector<int32_t> h_uoff, h_ul;         // U lists (CSR)
};

struct FmmPlan {
    // cache key
    int64_t key_n[3] = {0, 0, 0};
    const double *key_xy[3] = {nullptr, nullptr, nullptr};
    double alpha = 0;
    int opt_p = 0, opt_leaf = 0;
    double opt_tol = 0;

    // geometry
    double x0 = 0, y0 = 0, size = 0;  // bounding square
    int L = 0;                         // leaf level
    int lmin = 2;                      // coarsest level with M2L
    int p = 0, P = 0, Pp = 0;
    int64_t N = 0;
    int64_t toff[4] = {0, 0, 0, 0};    // type blocks in sorted order
    int nser = 0;                      // series terms for F_n at the leaf level
    int near_terms = 14;               // Horner length of the near-field series

    // sorted points
    DevBuf<double> px, py;
    DevBuf<float> pxf, pyf;            // leaf-centre-relative FP32 copies
    DevBuf<int32_t> perm;              // sorted position -> index within its set
    DevBuf<double> qs, dns, outs;      // sorted strengths and outputs
    DevBuf<float> qsf, dnsf;

    // boxes
    std::vector<LevelInfo> lev;
    int64_t nbox = 0, nleaf = 0;
    std::vector<uint32_t> hcode;       // Morton code per box (global index)
    std::vector<int32_t> hparent;
    DevBuf<double> bcx, bcy;           // centres
    DevBuf<int32_t> bparent;
    DevBuf<uint32_t> bcode;            // Morton code per box
    DevBuf<int32_t> fchild, nchild;    // first child (global index) and child count
    DevBuf<int32_t> slot_oid;          // [4 classes][27 slots] -> offset id in 0..39
    DevBuf<int32_t> child4;            // [nbox][4] child at each position, -1 if none
    DevBuf<int32_t> iota4;             // {0,1,2,3}: slot -> operator for M2M and L2L
    DevBuf<int32_t> iota40;            // 0..39: offset id -> M2L operator (sparse M2L)
    std::vector<int32_t> h_soid;       // host copy of slot_oid
    DevBuf<int4> up_tiles;             // M2M tiles: parents of levels lmin..L-1, 64 per tile
    DevBuf<int32_t> up_boxes;
    std::vector<int> up_tile_begin, up_tile_count;
    DevBuf<double> serc;               // [2][nser]: series coefficients of F_{p+1}, F_{p+2}
    DevBuf<int32_t> vlist;             // [nbox][27]
    DevBuf<int32_t> lrange;            // [nleaf][6] start/end per set (sorted positions)
    DevBuf<int32_t> ulist_off, ulist;  // CSR over leaves (leaf-local indices)
    std::vector<int32_t> h_lrange;     // host copy
    DevBuf<int32_t> pleaf;             // [N] leaf (level-local index) of every sorted point
    DevBuf<uint32_t> skeys;            // [N] sorted keys (set << 30 | Morton code at level 15)
    int64_t n_ulist = 0;               // U-list entries
    DevBuf<int32_t> dleaves;           // leaves (level-local) that hold dipole sources
    int64_t n_dleaves = 0;
    bool mq_kept = false;              // M's leaf level holds a charges-only pass's multipoles (keep_charge_m)
    // cached P2M rows: per charge [Pp], per dipole [2][Pp] (built on first use)
    DevBuf<double> p2m_rq, p2m_rd, p2m_gs;
    bool p2m_rows_built = false;

    // coefficients
    DevBuf<double> M, Lc;              // [nbox][Pp]
    DevBuf<float> Mf, Lf;

    // operators (double, column-major Pp x Pp blocks)
    DevBuf<double> m2m, l2l, m2l;      // [level][4][Pp*Pp], [level][4][Pp*Pp], [level][40][Pp*Pp]
    DevBuf<float> m2lf, l2lf;
    DevBuf<double> invFY, dipa, dipb;  // [level][p+2]
    DevBuf<double> cnn;                // 1/((n+1)(n+2)), n = 0 .. p+3

    std::map<int, std::unique_ptr<ActiveSet>> active;   // by target mask

    double build_ms = 0;
    // order check at build time (fmm_order.hip): the order first derived from
    // the tolerance and the largest sampled error of the order kept (-1: not run)
    int calib_p0 = 0;
    double calib_err = -1.0;
    double tables_ms = 0, check_ms = 0;   // host time of the operator tables, of the order check
    int mask_all() const {
        int m = 0;
        for (int s = 0; s < 3; ++s)
            if (toff[s + 1] > toff[s]) m |= 1 << s;
        return m;
    }
    // ---- adaptive tree (leaves at any level; U, V, W and X lists) ----
    // Leaf li is box leaf_box[li] (uniform tree: box lev[L].begin + li); the
    // leaf-indexed arrays above (lrange, pleaf, ulist) follow that numbering.
    bool adaptive = false;
    int opt_tree = 0;                              // 0 uniform, 1 adaptive, 2 automatic
    std::vector<int32_t> h_leaf_box, h_box_leaf;   // leaf -> box, box -> leaf (-1: split box)
    std::vector<int32_t> h_blevel;                 // level of every box
    DevBuf<int32_t> leaf_box, box_leaf, blevel, leaf_lev;
    DevBuf<uint32_t> leaf_start;                   // first level-15 cell of each leaf (sorted)
    DevBuf<int32_t> alr;                           // [nbox][6] leaf ranges by box (split boxes: empty)
    DevBuf<int32_t> p2m_list;                      // per level >= lmin: level-local indices of its leaves
    std::vector<int64_t> p2m_off;                  // [L + 2] slices of p2m_list by level
    std::vector<int64_t> up_off, up_n;             // per level: the split boxes' slice of up_boxes (M2M)
    DevBuf<int32_t> woff, wl, wleaves;             // W lists (CSR over leaves), leaves with a W list
    int64_t n_wl = 0, n_wleaves = 0;
    DevBuf<int32_t> xbox, xoff, xl;                // X lists: boxes with one, CSR of source leaves
    int64_t n_xbox = 0, n_xl = 0;
    std::vector<int32_t> h_xbox, h_xoff, h_xl;     // host copies
    int max_u = 0;                                 // longest U list
    // per-level tables for expansions at any level >= lmin
    int nser_stride = 0;                           // serc_lv: [level][2][nser_stride]
    std::vector<int> nser_lv;
    DevBuf<double> serc_lv, rI, invR_lv;           // rI: [level][p+3] = {I_0(R_l), I_n/I_{n-1} (n = 1..p+2)}
    DevBuf<int32_t> nser_dev;
    double near_tmax = 0;                          // largest t = r^2/(4 alpha^2) of a U-list pair

    bool fresh = false;
    uint64_t gen = 0;                  // unique per plan built in this process
    int last_mask = 0;
    int last_has_q = 0, last_has_d = 0;
};
FmmPlan *plan_in_slot(Context &ctx, int slot);

// tree.hip
void build_tree(Context &ctx, FmmPlan &pl, const SumProblem &pb);
// fmm_plan.cpp: boxes and lists from the sorted keys, then the translation
// operators and expansion tables of order p (rebuilt when p changes)
// (returns false, having built nothing, when the automatic form picks the
// adaptive tree for these points)
bool build_lists(Context &ctx, FmmPlan &pl, const std::vector<uint32_t> &keys, const uint32_t *dkeys);
// the adaptive tree (opt_tree 1): boxes split while they hold more than
// leaf_size points, then 2:1 balanced; U, V, W and X lists
void build_lists_adaptive(Context &ctx, FmmPlan &pl, const std::vector<uint32_t> &keys, const uint32_t *dkeys);
// lists.hip: the GPU parts of build_lists and get_active
void gpu_point_leaves(Context &ctx, FmmPlan &pl, const uint32_t *dkeys, const uint32_t *dleaf_codes);
void gpu_ulists(Context &ctx, FmmPlan &pl, const uint32_t *dleaf_codes);
void gpu_vlists(Context &ctx, FmmPlan &pl);
int64_t gpu_count_slots(Context &ctx, FmmPlan &pl, const int32_t *dboxes, int64_t n);
void gpu_point_leaves_adaptive(Context &ctx, FmmPlan &pl, const uint32_t *dkeys);
void gpu_ulists_adaptive(Context &ctx, FmmPlan &pl);
void gpu_wlists(Context &ctx, FmmPlan &pl, std::vector<int32_t> &woff, std::vector<int32_t> &wl);
void build_tables(Context &ctx, FmmPlan &pl, int p);
// terms of the near-field K0/K1 series for pairs with t = r^2/(4 alpha^2) <= tmax
int near_series_terms(double tmax);
// I_0(x) .. I_nmax(x) in extended precision
std::vector<long double> bessel_i_seq(long double x, int nmax);
// the stages between the leaf multipoles and the leaf local expansions
void fmm_m2m(Context &ctx, FmmPlan &pl);
void fmm_m2l(Context &ctx, FmmPlan &pl, ActiveSet &as, bool f32);
void fmm_l2l(Context &ctx, FmmPlan &pl, ActiveSet &as, bool f32);
// adaptive tree, after L2L: the W-list multipoles added into the sorted sums
// outs, then each leaf's local expansion at its points, written with outs to
// the caller's arrays out[set] (sets in mask)
void fmm_adaptive_finish(Context &ctx, FmmPlan &pl, int mask, double *outs, double *const out[3]);
ActiveSet &get_active(Context &ctx, FmmPlan &pl, int mask);
void ensure_near_layout(Context &ctx, FmmPlan &pl, ActiveSet &as);
// expansion orders with kernels: the smallest one >= p (at most kMaxOrder)
constexpr int kNumOrders = 7;
constexpr int kOrders[kNumOrders] = {8, 12, 16, 20, 24, 28, 31};
constexpr int kMaxOrder = 31;
int supported_order(int p);
int choose_order(double tol);

// fmm_order.hip: raises the order derived from fmm_tol until sampled outputs
// of probe strengths meet the tolerance (no-op when the order is given)
void calibrate_order(Context &ctx, FmmPlan &pl, const SumProblem &pb);

// fmm_kernels.hip
// bie (optional): the double-layer operator fused in (dn is then unused)
// parts: 1 the near field only, 2 the far field only, 3 both (the sums)
void fmm_run(Context &ctx, FmmPlan &pl, const double *q, const double *dn, double *const out[3],
             SumPrec prec, const BieFuse *bie = nullptr, int keep_charge_m = 0, int parts = 3);

// The tree of a slot for this problem (built, or rebuilt when stale).
FmmPlan &get_plan(Context &ctx, PlanSlot slot, const SumProblem &pb);

}  // namespace yk
