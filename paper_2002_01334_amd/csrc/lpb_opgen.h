// lpb_opgen.h -- host interface of the FP64 operator generator.
#pragma once
#include "lpb_internal.h"

namespace lpb {

struct OpgenInputs {
    int p;
    int n_ops, n_rkeys, n_rf;
    const OpDesc* d_ops;
    const RKey* d_rkeys;
    const FmmDev* d_fmm;
    const Medium* d_media;
    const int* d_free_list;
    int n_free;
    const int* d_react_list;
    int n_react;
    const int* d_rf_list;     // reaction FMM ids (n_rf)
    const int* d_rf_index;    // fmm id -> position in rf_list (-1 for free space)
    const double* d_btab;     // b^t_{nm} of the Legendre-product expansion
    const double* d_gtab;     // Gaunt integrals G(n,m;nu,mu;q)
    double* d_dtab;           // D_s table per reaction FMM (output)
    double* d_stab;           // scaled Sommerfeld integral tables per geometry key (output)
    double* d_pool;           // FP64 operators (output)
    float* d_pool32;          // FP32 copy (output, may be null)
    int* d_flag;              // bit 0: quadrature budget exceeded, bit 1: recurrence bound violated
    double quad_tol;
    // free-space M2L operators in the MFMA operand layout (KP x KP each)
    int KP;
    int n_swz;
    const int* d_swz_ops;
    double* d_swz64;          // FP64 mode
    float* d_swz32;           // mixed mode
    // canonical operators of the tiled levels for the orbit kernel (mixed
    // mode): rows in sign-class order (d_rowmap: row -> coefficient, -1 pad),
    // NRB 16-row blocks, same operand layout
    int n_orb, NRB;
    const int* d_orb_ops;
    const int* d_rowmap;
    float* d_orb32;
    // reaction point operators of adaptive trees (K doubles each at
    // PointOp::out): the points' offsets from their leaf centres (x, y, z;
    // with FP32 coordinates also the low parts), the leaf centres
    int n_pt;
    const PointOp* d_pt_ops;
    bool pt_f32;
    const void *t_u[6], *s_u[6];
    const double *tl_ctr, *sl_ctr;
    double* d_pt_vec;
};

hipError_t opgen_upload_constants();
hipError_t opgen_run(const OpgenInputs& in, hipStream_t st);
void gauss_legendre20(double* x, double* w);

}  // namespace lpb
