// Learned preconditioner: 3-D convolutional network inside flexible CG.
#include "common.h"

namespace ibm {

int cnn_fcg_solve(ibm_ctx* c, const double* b, double* x, const ibm_solver_opts* o, ibm_stats* st, hipStream_t s) {
    (void)b; (void)x; (void)o; (void)st; (void)s;
    if (!c->cnn) {
        set_error("IBM_SOLVER_FCG_CNN: no network attached to the context");
        return IBM_ERR_ARG;
    }
    set_error("IBM_SOLVER_FCG_CNN: not available");
    return IBM_ERR_ARG;
}

}  // namespace ibm
