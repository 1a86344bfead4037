// Pieces of the C ABI shared by the single-call entry points (api.cpp) and
// the request loop (server.cpp).
#pragma once

#include <stdint.h>

#include <new>
#include <string>
#include <vector>

#include "engine.h"
#include "sdbg.h"

namespace sdbg_abi {

extern thread_local std::string t_err;

// Runs f, turning exceptions into an error code and the thread's message.
template <typename F>
int guarded(F&& f) {
  try {
    t_err.clear();
    return f();
  } catch (const sdbg::Error& e) {
    sdbg::prof_flush();
    t_err = e.what();
    return e.code;
  } catch (const std::bad_alloc&) {
    t_err = "host allocation failed";
    return SDBG_E_NOMEM;
  } catch (const std::exception& e) {
    t_err = e.what();
    return SDBG_E_HIP;
  }
}

// Object kinds of the registry (sdbg_free releases any registered object).
enum ObjKind { kEdges = 1, kGraph = 2, kIndex = 3, kUnitigs = 4, kBwt = 5 };
void reg_add(void* p, int kind);
int reg_kind(const void* p);
void free_index(void* p);    // navigation index (nav.hip)
void free_unitigs(void* p);  // unitig set (nav.hip)
void free_bwt(void* p);      // read-set BWT (bwt.hip)

void check_k(uint32_t k);
void check_params(const sdbg_params* p);
void pool_free(void* p);
// Library objects (registered, so that sdbg_free accepts them).
sdbg_edges* wrap_edges(const sdbg::EdgesOut& eo, uint32_t k);
sdbg_graph* wrap_graph(const sdbg::GraphOut& go, uint32_t k);
std::vector<uint64_t> host_offsets(sdbg::Ctx& c, const sdbg_reads* r);
uint64_t occ_bound(const std::vector<uint64_t>& o, uint32_t k);
uint64_t device_budget(const sdbg_params* p);

}  // namespace sdbg_abi
