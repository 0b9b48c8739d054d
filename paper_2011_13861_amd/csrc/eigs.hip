// Block eigensolver (placeholder until the solver lands).
#include "kl_internal.h"

extern "C" kl_status kl_eigs(kl_problem *P, const kl_eigs_opts *opts, const double *x0,
                             int32_t nvec0, double *evals, double *evecs, int64_t ldv,
                             kl_eigs_report *rep) {
    (void)P; (void)opts; (void)x0; (void)nvec0; (void)evals; (void)evecs; (void)ldv; (void)rep;
    kl::set_error("kl_eigs: not available yet");
    return KL_EINVAL;
}
