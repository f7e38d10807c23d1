// Layout helpers shared by every kernel variant and the C ABI.
#include "xkp_internal.h"

namespace xkp {

WsLayout ws_layout(int nmax, int mmax, int npad) {
    auto up = [](size_t v) { return (v + 63) & ~(size_t)63; };
    WsLayout L;
    L.npad = npad;
    L.v = 0;
    L.cE = up((size_t)basis_ldv(nmax) * (mmax + 1));
    L.cW = L.cE + up(L.npad);
    L.cN = L.cW + up(L.npad);
    L.cS = L.cN + up(L.npad);
    L.c32 = L.cS + up(L.npad);
    L.w = L.c32 + up(2 * (size_t)L.npad);
    L.stride = L.w + up((size_t)basis_ldv(nmax) * (mmax + 1));
    return L;
}

size_t basis_off_v() { return 256; }
int basis_ldv(int n) { return (n + 8) & ~7; }
size_t basis_bytes(int n, int m) {
    size_t o = basis_off_vb(n, m) + 2 * (size_t)basis_ldv(n) * (m + 1);
    return (o + 255) & ~(size_t)255;
}

}  // namespace xkp
