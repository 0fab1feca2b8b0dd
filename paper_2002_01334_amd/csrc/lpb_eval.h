// lpb_eval.h -- argument block of the evaluation kernels.
#pragma once
#include "lpb_internal.h"

namespace lpb {

template <typename T>
struct EvalArgs {
    int p, K, nslots;
    int KP;             // padded coefficient stride of ME/LE rows (multiple of 16, >= K)
    int64_t ncharges;
    int64_t near_off;           // start of the free-space near-field slot in parts (after the component slots)
    const FmmDev* fmm;
    const Medium* media;
    // sources (sorted by FMM, leaf)
    int n_src;
    const int* s_cidx;
    const T *s_ux, *s_uy, *s_uz;
    const T *s_lx, *s_ly, *s_lz;   // FP32: low parts (u - (double)hi) of the offsets; FP64: null
    T* qs;
    const double* q;
    const int *sl_start, *sl_me, *sl_fmm;
    const double *sl_h, *sl_ctr;
    // targets
    const T *t_ux, *t_uy, *t_uz;
    const T *t_lx, *t_ly, *t_lz;
    const int *t_cidx, *t_out;
    const int *tl_start, *tl_le, *tl_fmm;
    const double *tl_h, *tl_ctr;
    // expansions: n_me (n_le) rows of KP, plus a zero row at index n_me (n_le)
    T* me;
    T* le;
    int n_le, n_me;
    // work lists
    const int *p2m_leaves, *l2p_leaves, *p2p_free_leaves;
    const int* p2p_free_t0;     // first target of each free near-field work item
    const int* p2p_free_ts;     // its target count T (<= 64) | source splits S << 8 (T S <= 64 lanes)
    const int *m2l_boxes, *m2l_ptr, *m2l_src, *m2l_op;
    const int* m2l_xc;          // per untiled V-list pair: result transform (0..7 reflection, kXfRotate + dir rotation)
    // batched translations (M2M, L2L, untiled V-list pairs): see Plan
    const int *bw_term_ptr, *bw_op, *bw_src, *bw_dst;
    const int* bw_xc;           // per column transform code (-1 none, 0..7 reflection, kXfRotate + dir rotation)
    const T* rot_tab;           // [kXfDirs][p+1][2]: cos, sin (m phi) of each V-list direction
    const T* xf_ab;             // [kXfRotate + kXfDirs][K][2]: (a, b) with row' = a row + b partner row,
                                //   the frame change of each transform code per coefficient row
    T* m2l_scratch;     // one row of K per untiled V-list pair
    const int *p2p_ptr, *p2p_src;
    const int *rp_ptr, *rp_fmm, *rp_src;   // reaction near field: per target leaf, (FMM, source leaf)
    int n_react_targets;
    const int *react_tgt_leaf, *react_tgt_slot;
    const double *gl_x, *gl_w;
    double quad_tol;
    double* parts;
    double* phi;
    // tiled free-space M2L
    int n_tiles;
    const Tile* tiles;
    const TileFL* tfl;
    const int *grid_me, *grid_le, *optab, *oct_codes;
    const T* pool_swz;          // operators in the MFMA operand layout, KP x KP each
    const T* refl_sign;         // [8][KP]: diagonal of D for each reflection code (padding rows +1)
    // solid-harmonic recurrence coefficients (packed (n,m) index):
    //   R_m^m = amm[m] (x+iy)^m, R_n^m = alpha z R_{n-1}^m - beta |v|^2 R_{n-2}^m
    const T *sh_amm, *sh_alpha, *sh_beta;
    // Bessel-ratio tables (FP64): p-dependent recurrence/series factors, and
    // 1/it_n(lam h) per FMM and level for the source (ith_s) and target (ith_t) lambda
    const double *bes_tab, *ith_s, *ith_t;
    const int* swz_index;       // op -> position in pool_swz
    // tiled M2L by reflection orbits (FP32, p >= kOrbitMinP): orbit table
    // (see kOrbits), op -> canonical operator position in pool_orb (rows in
    // sign-class order), and operand row -> coefficient (-1 padding)
    const int *orb_tab, *orb_index, *orb_rows;
    const int* orb_kcls;        // sign class of each coefficient (KP entries, padding 0)
    const T* pool_orb;
    // block -> work schedules of the matrix-core kernels (see sched_index)
    int tile_sched, batch_sched;
    // leaf levels (the scale of a leaf's expansion), and the W- and X-lists
    // of adaptive trees (see Plan): target leaves with W entries, X target
    // boxes, reaction point operators (K doubles each)
    const int *sl_lv, *tl_lv;
    int n_w_leaves, n_x_boxes;
    const int* w_leaves;
    const int *w_ptr, *w_fmm, *w_me, *w_lv;
    const double* w_ctr;
    const int64_t* w_vec;
    const int *x_box_le, *x_box_lv, *x_box_ptr;
    const double* x_box_ctr;
    const int *x_fmm, *x_sl;
    const int64_t* x_vec;
    const double* pt_vec;
    // 4 pi i_n(lam h) per FMM and level (source-side lambda for M2P, target
    // side for P2L), (kMaxDepth + 1) x (LPB_MAX_P + 1) per FMM, and the
    // solid-harmonic recurrence coefficients in FP64 (amm[p+1], alpha[Kp], beta[Kp])
    const double *fin_s, *fin_t, *sh64;
};

struct EvalSched {
    int n_p2m, n_l2p, n_p2p_free, n_m2l_boxes;
    int p2m_nl = 2, l2p_nl = 2;   // leaves per 64-lane block of the fixed-order P2M / L2P (2 or 4)
    int bm2m_lv[kMaxDepth + 2];
    int bl2l_lv[kMaxDepth + 2];
    int bm2l_w0, bm2l_w1;
};

// A second stream for the untiled V-list translations, which then run beside
// the tiled M2L (they write other LE boxes): `fork` is recorded on the main
// stream before them, `join` on the side stream after them.  A third stream
// takes the free-space near field, which writes a slot of its own and so runs
// beside the whole far field (`near_fork` after the charges are gathered and
// the slots cleared, `near_join` before the slots are summed).
struct EvalFork {
    hipStream_t side = nullptr;
    hipEvent_t fork = nullptr, join = nullptr;
    hipStream_t near = nullptr;
    hipEvent_t near_fork = nullptr, near_join = nullptr;
};

// One evaluation.  With per-stage events (ev) or without a fork every pass
// runs on st in order.
template <typename T>
hipError_t eval_run(const EvalArgs<T>& A, const EvalSched& S, int stages, hipStream_t st, hipEvent_t* ev,
                    const EvalFork* fk = nullptr);

// Launchers of kernels that live in their own translation units: the tiled
// free-space M2L (all forms) and P2M / L2P with the order fixed at compile
// time (FP32, 2 <= p <= 15; nothing is launched for other p).
template <typename T>
void launch_m2l_tile(const EvalArgs<T>& A, hipStream_t st);
template <int P>
void launch_m2l_orbit_p(const EvalArgs<float>& A, hipStream_t st);   // kOrbitMinP <= P <= kOrbitMaxP
template <typename T>
bool launch_m2l_tile_kb(const EvalArgs<T>& A, bool wide, hipStream_t st);
// W-list M2P and X-list P2L of adaptive trees (nothing is launched without them)
template <typename T>
void launch_m2p(const EvalArgs<T>& A, hipStream_t st);
template <typename T>
void launch_p2l(const EvalArgs<T>& A, hipStream_t st);
// (nl = 2 or 4 leaves per 64-lane block)
void launch_p2m_fixed(const EvalArgs<float>& A, int n_leaves, int nl, hipStream_t st);
void launch_l2p_fixed(const EvalArgs<float>& A, int n_leaves, int nl, hipStream_t st);

// One matrix-core stage alone, for schedule tuning: which = 0 the tiled M2L,
// 1 the batched translations (M2M, untiled M2L, L2L).  Leaves ME/LE/scratch
// contents that the next full evaluation overwrites.
template <typename T>
hipError_t stage_run(const EvalArgs<T>& A, const EvalSched& S, int which, hipStream_t st);

}  // namespace lpb
