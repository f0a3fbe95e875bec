// Helpers shared by the host-side C ABI sources.
#pragma once

#include <stdarg.h>
#include <stdint.h>

#include "ge.h"

namespace ge {

// Record a printf-style message as the calling thread's last error and
// return `st`.
ge_status set_error(ge_status st, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
ge_status vset_error(ge_status st, const char *fmt, va_list ap);

// Coefficients of the scheme for mesh ratio r, evaluated on the host in FP64
// by the same expressions for every entry point (single rod and batch), so
// both paths feed the kernels identical values.
struct SchemeCoef {
    double c1, c2, cs;   // (r+r^2)/(1+2r), r^2/(1+2r), r/(1+r)
};
SchemeCoef scheme_coef(double r);

int64_t comp_offset(int64_t n);

// Rod count, points per rod and precision of a batch plan; false for NULL.
bool batch_shape(ge_batch_t b, int64_t *nrods, const int64_t **n, int *prec);

// Status words a plan's kernels may raise (StatusWord in ge_level.h): pinned,
// mapped host memory, written by the kernels with plain stores and read by
// the host without waiting for the device.  `dev` is the kernels' view.
// Without a usable device the allocation fails and both pointers stay null.
struct StatusWords {
    int *host = nullptr;
    int *dev = nullptr;
};
bool status_alloc(StatusWords &w);
// Waits for the device (a kernel may still hold the pointer) and frees.
void status_free(StatusWords &w);
// True (and the word cleared) if a finished launch raised word `word`.
bool status_take(StatusWords &w, int word);

// Message recorded by the last set_error on the calling thread.
const char *last_error_str();

}  // namespace ge
