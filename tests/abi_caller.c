/* A plain C caller of the library (test infrastructure): includes only the
 * public header, links libasaga.so, and solves a 6 x 4 logistic problem in
 * serial mode from host arrays.  Prints the objective and x after 25 epochs
 * (17 significant digits) so that a test can compare them with the oracle.
 * Exit status: 0 on success, 1 if a call failed (its message is printed). */
#include <stdio.h>

#include "asaga.h"

int main(void) {
    const int64_t rowptr[] = {0, 2, 3, 5, 7, 8, 10};
    const int32_t colidx[] = {0, 2, 1, 0, 3, 1, 2, 3, 0, 1};
    const double val[] = {0.6, -0.8, 1.0, 0.28, 0.96, -0.6, 0.8, 1.0, 0.8, 0.6};
    const double b[] = {1.0, -1.0, 1.0, 1.0, -1.0, -1.0};
    asaga_problem p = {0};
    p.n = 6;
    p.d = 4;
    p.rowptr = rowptr;
    p.colidx = colidx;
    p.val = val;
    p.b = b;
    p.lambda = 0.1;
    p.val_dtype = ASAGA_VAL_F64;
    p.loss = ASAGA_LOSS_LOGISTIC;
    p.mem = ASAGA_MEM_HOST;
    asaga_opts o = {0};
    o.mode = ASAGA_MODE_SERIAL;
    o.seed = 3;
    asaga_ctx* c = NULL;
    if (asaga_init(&c, &p, &o) != ASAGA_OK) {
        printf("asaga_init: %s\n", asaga_last_error(NULL));
        return 1;
    }
    double f = 0.0, x[4];
    if (asaga_epochs(c, 25) != ASAGA_OK || asaga_objective(c, 0, NULL, &f) != ASAGA_OK ||
        asaga_get_x(c, 0, x) != ASAGA_OK) {
        printf("call failed: %s\n", asaga_last_error(c));
        asaga_free(c);
        return 1;
    }
    printf("%.17g %.17g %.17g %.17g %.17g\n", f, x[0], x[1], x[2], x[3]);
    asaga_free(c);
    return 0;
}
