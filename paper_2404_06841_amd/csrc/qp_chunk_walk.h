// Walk of the stiffness product over its mode records (plain C++, also
// compiled on the host by the tests).
//
// A product gathers the neighbour values of its g modes chunk by chunk, each
// chunk a compile-time count of records: records [0, gp), gp = g rounded up
// to a multiple of 4 (the records staged in LDS; the padding ones read
// zero).  The walk takes chunks of KC records while they fit, then one chunk
// of KC / 2 when that keeps the start a multiple of 4, then chunks of 4 up
// to gp.  A chunk running past gp would read records that were never staged.
#pragma once

namespace qp {

// whether the walk takes a chunk of KC / 2 records at record rb
constexpr bool take_half_chunk(int KC, int rb, int gp)
{
    return KC / 2 >= 4 && (KC / 2) % 4 == 0 && rb + KC / 2 <= gp;
}

// where the walk over gp records ends (gp when every chunk stays inside)
constexpr int chunk_walk_end(int KC, int gp)
{
    int rb = 0;
    while (rb + KC <= gp) rb += KC;
    if (take_half_chunk(KC, rb, gp)) rb += KC / 2;
    while (rb < gp) rb += 4;
    return rb;
}

// whether the walk ends exactly at gp for every gp = 4, 8, ..., gpmax
constexpr bool chunk_walk_exact(int KC, int gpmax)
{
    if (KC < 4 || KC % 4 != 0) return false;
    for (int gp = 4; gp <= gpmax; gp += 4)
        if (chunk_walk_end(KC, gp) != gp) return false;
    return true;
}

}  // namespace qp
