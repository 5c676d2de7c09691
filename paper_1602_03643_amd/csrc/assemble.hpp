// Assembly and small vector helpers shared with the IPCS step.
#pragma once

#include "internal.hpp"

namespace oasis {

struct P3 {
    const double *p[3];
};

int check_csr(const oasis_csr *A);
int check_mesh_colored(const oasis_mesh *m);

// out += alpha * form, colour by colour; CONV uses u_bar = c1 U1 + c2 U2.
// missing (device int, nullable) is set when an element entry has no slot.
int assemble_colored(hipStream_t s, const oasis_mesh *m, const int *rp, const int *ci, double *out,
                     int form, double alpha, P3 U1, P3 U2, double c1, double c2, int *missing);

// y = a * x (x == nullptr: y = 0)
int scale_copy(hipStream_t s, long long n, double *y, const double *x, double a);


}  // namespace oasis
