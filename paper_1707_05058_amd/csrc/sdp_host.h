// Host-only pieces of libsdp shared by the C ABI (sdp_api.cpp) and the
// validation (sdp_validate.cpp): the error type that carries a status code
// to the ABI boundary, and the index structures built from one instance.
// Plain C++ with no HIP dependency, so the validation also builds and runs
// under the host sanitizers.
#pragma once

#include <cstdint>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/sdp.h"

namespace sdp_host {

struct SdpError : std::runtime_error {
  int code;
  SdpError(int c, const std::string &m) : std::runtime_error(m), code(c) {}
};

[[noreturn]] inline void fail(int code, const std::string &msg) { throw SdpError(code, msg); }

inline int64_t round_up(int64_t x, int64_t a) { return (x + a - 1) / a * a; }

// One instance after validation: host-side index structures.
struct HostInst {
  const sdp_instance *src;
  int32_t n, m, p, fmt, ld, ldm;
  int64_t nnz;
  std::vector<int32_t> blk_loc;     // packed entries of all cliques -> local coordinate
  std::vector<int64_t> cl_off;      // packed offset of each clique (local)
  std::vector<int32_t> D;           // overlap counts
  int64_t npk;
};

// Checks one instance (pattern sorted and lower with every diagonal, cliques
// in natural order and covering the pattern, finite data, cliques of at most
// max_clique vertices) and builds its entry selectors (Section 4: packed
// block entry (a, b) of clique k is pattern coordinate (v_a, v_b)) and the
// overlap counts D = sum_k H_k^T H_k.  Throws SdpError with the status code.
int validate_and_index(const sdp_instance &I, int max_clique, HostInst &H);

}  // namespace sdp_host
