// Host build of the double-double E = e^{i zeta} used by the node preparation
// (the same header the device code includes), for the CPU test against
// high-precision decimal arithmetic.
#include "../paper_2108_01786_amd/csrc/ddmath.h"

extern "C" void dd_expi_host(double x, double y, double *out) {
    wwbi::DD er, ei;
    wwbi::dd_expi(x, y, er, ei);
    out[0] = er.hi;
    out[1] = er.lo;
    out[2] = ei.hi;
    out[3] = ei.lo;
}
