// Walk of the stiffness product over its mode records (plain C++, also
// compiled on the host by the tests).
//
// A product gathers the neighbour values of its g modes chunk by chunk, each
// chunk a compile-time count of records, in record order: chunks of KC
// records while they fit, then one chunk of KC / 2 (when that is at least 4
// and fits), then chunks of 4, then one chunk of the 1 to 3 records left.
// The walk ends exactly at record g: the records staged past g (zero-weight
// padding up to a multiple of 4) are never gathered, and no chunk reads a
// record that was not staged.
#pragma once

#include <type_traits>

namespace qp {

// chunk(std::integral_constant<int, C>(), rb) for each chunk [rb, rb + C)
template <int KC, typename F>
__attribute__((always_inline)) constexpr void walk_records(int g, F &&chunk)
{
    static_assert(KC >= 4 && KC % 4 == 0, "full chunks are whole groups of four records");
    int rb = 0;
    for (; rb + KC <= g; rb += KC) chunk(std::integral_constant<int, KC>(), rb);
    if constexpr (KC / 2 >= 4) {
        if (rb + KC / 2 <= g) {
            chunk(std::integral_constant<int, KC / 2>(), rb);
            rb += KC / 2;
        }
    }
    for (; rb + 4 <= g; rb += 4) chunk(std::integral_constant<int, 4>(), rb);
    switch (g - rb) {
    case 3: chunk(std::integral_constant<int, 3>(), rb); break;
    case 2: chunk(std::integral_constant<int, 2>(), rb); break;
    case 1: chunk(std::integral_constant<int, 1>(), rb); break;
    default: break;
    }
}

}  // namespace qp
