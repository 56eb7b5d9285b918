// Shared host-side helpers of libhplmm: error text, status plumbing.
#pragma once

#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "../../include/hplmm.h"

namespace hplmm {

void set_error(const std::string &msg);

struct Error {
    hplmm_status code;
    std::string msg;
};

// Throw inside the library; the C ABI converts to a status code.
[[noreturn]] void fail(hplmm_status code, const std::string &msg);

template <class F>
hplmm_status guarded(F &&f) {
    try {
        return f();
    } catch (const Error &e) {
        set_error(e.msg);
        return e.code;
    } catch (const std::bad_alloc &) {
        set_error("host allocation failed");
        return HPLMM_E_OOM;
    } catch (const std::exception &e) {
        set_error(e.what());
        return HPLMM_E_ARG;
    }
}

// Free-node numbering of a voxel solid: nodes touched by a solid voxel, not
// on the plane z = 0, ascending lattice id (x fastest).
struct NodeMap {
    int32_t nx = 0, ny = 0, nz = 0;
    int64_t NX = 0, NY = 0, NZ = 0;
    std::vector<int32_t> lat2free;   // lattice id -> free id or -1
    std::vector<int64_t> free2lat;   // free id -> lattice id
    void build(int32_t nx_, int32_t ny_, int32_t nz_, const uint8_t *solid);
    int64_t lat(int64_t i, int64_t j, int64_t k) const { return i + NX * (j + NY * k); }
    int64_t n() const { return (int64_t)free2lat.size(); }
};

// Element stiffness of the unit-cube Q1 hexahedron for E = 1, Poisson nu.
// Local node a sits at corner (a&1, a>>1&1, a>>2&1); dof 3a + c.
void q1_element_stiffness(double nu, double K[24][24]);

}  // namespace hplmm
