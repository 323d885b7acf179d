// k_vjp.hip -- vector-Jacobian product of the accelerations (placeholder
// until the backward kernels land).
#include "rcb_internal.h"

namespace rcb {

rcb_status gravity_vjp(rcb_tree *t, const void *gx, const void *gy, const void *gz, void *dx,
                       void *dy, void *dz, void *dm, hipStream_t s) {
    (void)t; (void)gx; (void)gy; (void)gz; (void)dx; (void)dy; (void)dz; (void)dm; (void)s;
    set_error("rcb_gravity_vjp: not implemented");
    return RCB_ESTATE;
}

}  // namespace rcb
