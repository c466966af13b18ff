// hsga_host.hpp -- host-side pieces shared by the run API (hsga_api.cpp)
// and the batched / served pool (hsga_pool.cpp).  Not part of the public
// interface.
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "../../include/hsga.h"
#include "hsga_device.hpp"
#include "hsga_internal.hpp"

struct ga_run {
    ga_config cfg;
    uint32_t I, A, N, S, SW;
    hipStream_t stream;
    uint32_t* trait[2];
    uint32_t* counter[2];
    uint32_t* surf[2];
    uint32_t* outbox[2];
    uint32_t* layout;
    uint32_t* sites;     // synchronous: the site schedule of a launch batch
    hsga::RuleTable* rules;   // the site rule's tables (device)
    uint32_t* ring;      // asynchronous: sites of the latest kSiteRing ingests
    uint32_t ring_hi;    // asynchronous: ingests below this are in the ring (the
                         // last kSiteRing of them)
    uint32_t gens;       // site schedule capacity
    uint32_t T;          // generations (ticks, when asynchronous) enqueued
    uint64_t horizon;
    uint32_t apt;        // agents per thread (1, 2, 4; divides N)
    uint32_t block;      // workgroup threads
    bool timing;
    bool pooled = false; // a slot of a pool (its generation targets live there)
    bool resident = true;  // a synchronous run that fits one workgroup steps resident
    bool broken = false; // a ga_step failed after enqueueing part of its work
    struct Span { hipEvent_t start, stop; uint32_t launches; };
    std::vector<Span> spans;
    std::vector<hipEvent_t> spare;
};

namespace hsga_host {

constexpr uint32_t kDefaultGens = 4096;
constexpr size_t kAlign = 256;
constexpr size_t kMaxStepLds = 65536;
// Largest run that steps in the resident form (one workgroup for the whole
// torus): past this many agents the generation's births on one CU take
// longer than a launch over many CUs.
constexpr uint32_t kResidentMaxAgents = 4096;

int fail(int status, const std::string& msg);
int hip_fail(hipError_t e, const char* what);
const char* last_error();
inline size_t align_up(size_t x) { return (x + kAlign - 1) & ~(kAlign - 1); }

struct Carve {
    size_t trait, counter, surf, outbox, layout, rules, sites, total;
};

// Enqueue the upload of the site rule's tables of a surface (one, or two
// for hybrid) to dev on stream, from pinned host copies the library keeps.
hipError_t upload_tables(uint32_t kind, uint32_t S, hsga::RuleTable* dev, hipStream_t stream);

// Surface words per agent of a validated config.
inline uint32_t surface_words(const ga_config& c) {
    return c.surface_sites * c.differentia_bits / 32;
}

// Byte offsets of each buffer of a run of a validated config in its arena.
// Only asynchronous runs keep counter planes: in a synchronous run every
// counter is the generation count (counter == 0 and no bytes then).  A
// synchronous run's `sites` holds a launch batch's site schedule (gens
// words); an asynchronous run's holds the site rule's tables and a ring of
// the sites of its latest ingests instead.
Carve carve(const ga_config& cfg, uint32_t gens);

// GA_OK, or GA_EINVAL with the reason in ga_last_error().
// Check a caller's config (either accepted struct_size) and, if out is not
// NULL, store it in the current layout with absent fields zero.
int validate(const ga_config* in, ga_config* out);

// Fill r for cfg over the arena at base (already checked to hold
// carve(...).total bytes) and enqueue the founders.
int run_init(ga_run* r, const ga_config* cfg, uint8_t* base, uint32_t gens, hipStream_t stream);

inline uint32_t tile_islands(uint32_t block, uint32_t apt, uint32_t N) { return block * apt / N; }

// Enqueue the run's layout after the ingests of generation (tick) count T
// (closed form of the site rule, written by a kernel).
int set_run_layout(ga_run* r, uint32_t T);

// Parameters of generation g of a run whose current site schedule starts
// at ingest tau0.
hsga::StepParams step_params(const ga_run* r, uint32_t g, uint32_t tau0);

// hsga::BirthModel of a configuration.
uint32_t birth_model(const ga_config& cfg);

}  // namespace hsga_host
