// Index tables of the packed symmetric moment components and of the
// invariant feature order (device constant memory and host copies).
//
// Packed components of one radial channel (20 values):
//   0        Psi0
//   1..3     Psi1: x y z
//   4..9     Psi2: xx xy xz yy yz zz
//   10..19   Psi3: xxx xxy xxz xyy xyz xzz yyy yyz yzz zzz
// Full (unpacked) layout of one channel in LDS (40 values):
//   0 Psi0 | 1..3 Psi1[a] | 4..12 Psi2[a][b] | 13..39 Psi3[a][b][c]
//
// Invariant families and their first feature (S = 5, F = 360):
//   fam1  Psi0[s1]                                     offset   0  (5)
//   fam2  Psi1[s1]_a Psi1[s2]_a            s1<=s2     offset   5  (15)
//   fam3  Psi2[s1]_ab Psi2[s2]_ab          s1<=s2     offset  20  (15)
//   fam4  Psi3[s1]_abc Psi3[s2]_abc        s1<=s2     offset  35  (15)
//   fam5  tr(Psi2[s1] Psi2[s2] Psi2[s3])   s1<=s2<=s3 offset  50  (35)
//   fam6  Psi1[s1]_a Psi1[s2]_b Psi2[s3]_ab s1<=s2    offset  85  (75)
//   fam7  Psi2[s1]_ab Psi3[s2]_acd Psi3[s3]_bcd s2<=s3 offset 160 (75)
//   fam8  Psi1[s1]_a Psi3[s2]_abc Psi2[s3]_bc         offset 235 (125)
// Inside a family the index tuples run lexicographically, last fastest.
#pragma once

namespace gmnn {

constexpr int kS = 5;          // radial channels supported by the kernels
constexpr int kPacked = 20;    // packed components per channel
constexpr int kFull = 40;      // full components per channel
constexpr int kF = 360;        // invariants for S = 5
constexpr int kFP = 384;       // invariants padded to a multiple of 32

constexpr int kFam2 = 5, kFam3 = 20, kFam4 = 35, kFam5 = 50, kFam6 = 85, kFam7 = 160, kFam8 = 235;

// full index r (0..39) -> packed index
__constant__ static const unsigned char c_full_to_packed[kFull] = {
    0, 1, 2, 3,
    // Psi2[a][b], a,b in 0..2
    4, 5, 6, 5, 7, 8, 6, 8, 9,
    // Psi3[a][b][c]
    10, 11, 12, 11, 13, 14, 12, 14, 15,   // a = 0
    11, 13, 14, 13, 16, 17, 14, 17, 18,   // a = 1
    12, 14, 15, 14, 17, 18, 15, 18, 19};  // a = 2

// packed index -> number of full entries it stands for, and their full indices
__constant__ static const unsigned char c_packed_mult[kPacked] = {1, 1, 1, 1, 1, 2, 2, 1, 2, 1,
                                                                  1, 3, 3, 3, 6, 3, 1, 3, 3, 1};
__constant__ static const unsigned char c_packed_full[kPacked][6] = {
    {0}, {1}, {2}, {3},
    {4}, {5, 7}, {6, 10}, {8}, {9, 11}, {12},
    {13}, {14, 16, 22}, {15, 19, 31}, {17, 23, 25}, {18, 20, 24, 28, 32, 34}, {21, 33, 37},
    {26}, {27, 29, 35}, {30, 36, 38}, {39}};

// pair index p (0..14) <-> (s1 <= s2)
__constant__ static const unsigned char c_pair_s1[15] = {0, 0, 0, 0, 0, 1, 1, 1, 1, 2, 2, 2, 3, 3, 4};
__constant__ static const unsigned char c_pair_s2[15] = {0, 1, 2, 3, 4, 1, 2, 3, 4, 2, 3, 4, 3, 4, 4};
__constant__ static const unsigned char c_pair_index[5][5] = {
    {0, 1, 2, 3, 4}, {1, 5, 6, 7, 8}, {2, 6, 9, 10, 11}, {3, 7, 10, 12, 13}, {4, 8, 11, 13, 14}};

// sorted triple index t (0..34) <-> (s1 <= s2 <= s3); c_tri_index takes any order
__constant__ static const unsigned char c_tri_s1[35] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 2, 2, 2, 2, 2, 2, 3, 3, 3, 4};
__constant__ static const unsigned char c_tri_s2[35] = {0, 0, 0, 0, 0, 1, 1, 1, 1, 2, 2, 2, 3, 3, 4, 1, 1, 1, 1, 2, 2, 2, 3, 3, 4, 2, 2, 2, 3, 3, 4, 3, 3, 4, 4};
__constant__ static const unsigned char c_tri_s3[35] = {0, 1, 2, 3, 4, 1, 2, 3, 4, 2, 3, 4, 3, 4, 4, 1, 2, 3, 4, 2, 3, 4, 3, 4, 4, 2, 3, 4, 3, 4, 4, 3, 4, 4, 4};
__constant__ static const unsigned char c_tri_index[5][5][5] = {
    {{0, 1, 2, 3, 4}, {1, 5, 6, 7, 8}, {2, 6, 9, 10, 11}, {3, 7, 10, 12, 13}, {4, 8, 11, 13, 14}},
    {{1, 5, 6, 7, 8}, {5, 15, 16, 17, 18}, {6, 16, 19, 20, 21}, {7, 17, 20, 22, 23}, {8, 18, 21, 23, 24}},
    {{2, 6, 9, 10, 11}, {6, 16, 19, 20, 21}, {9, 19, 25, 26, 27}, {10, 20, 26, 28, 29}, {11, 21, 27, 29, 30}},
    {{3, 7, 10, 12, 13}, {7, 17, 20, 22, 23}, {10, 20, 26, 28, 29}, {12, 22, 28, 31, 32}, {13, 23, 29, 32, 33}},
    {{4, 8, 11, 13, 14}, {8, 18, 21, 23, 24}, {11, 21, 27, 29, 30}, {13, 23, 29, 32, 33}, {14, 24, 30, 33, 34}}};

}  // namespace gmnn
