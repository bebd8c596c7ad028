// Internal definitions shared by the translation units of liblbm_axi.so.
#pragma once

#include "axi_device.hpp"
#include "axi_half.hpp"
#include "../../include/lbm_axi.h"

#include <stddef.h>

namespace axi {

constexpr int TZ = 64;          // tile width along z: one wave per tile row
#ifndef AXI_PLANE_PAD
#define AXI_PLANE_PAD 64
#endif
constexpr int PLANE_PAD = AXI_PLANE_PAD;   // spare elements per population plane

} // namespace axi

// One case: its geometry, rates and the pointers into its device block.
struct lbm_axi_case {
    lbm_axi_params prm;
    hipStream_t stream;
    char *base;
    size_t bytes;
    int64_t t;
    int cur;               // ping-pong buffer holding the current state
    int tile_r;
    int device;            // HIP device the case was initialised on
    axi::Geom geom;             // geometry of the step launch (tiles for tile_r)
    axi::Phys<double> P64;
    axi::Phys<float> P32;
    axi::Codec codec;      // FP16-deviation storage scales
    size_t esize;          // bytes per stored value (FP16-deviation: 2)
    void *pop[2][2];       // [buffer][f or g]
    void *aux;
    double *fld;
    double *part;          // per-workgroup partials of the diagnostics reductions
    lbm_axi_diag *diag;    // the diagnostics record, reduced on the device
};

namespace axi {
// geometry of the step launch for a given tile height
Geom geom_for(const lbm_axi_case *c, int tile_r);
// elements between population planes of an nr x nz case
int64_t plane_elems(int nr, int nz);
// FP16-deviation storage: buffers of ping-pong side b, and the step from side cur
struct HalfBuf {
    float *f0;       // f_0 plane (FP32)
    half_t *f;       // f_1..f_8 planes (FP16), plane p at f + (p - 1) * plane
    half_t *g;       // g_0..g_8 planes (FP16)
    float *phi;      // stored phase field of side b
};
HalfBuf half_buf(const lbm_axi_case *c, int b);
HalfState half_state(const lbm_axi_case *c, int cur);
} // namespace axi
