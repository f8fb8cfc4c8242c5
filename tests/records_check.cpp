// Host program: the qubit shared-list record helpers (qram_records.h) on
// hand-built records, including records whose count word is damaged.  A
// damaged count must raise ERR_LIST and must not make a helper write outside
// the address's records.  Prints "ok" and exits 0 when every check passes.
#include <cstdio>
#include <cstring>
#include <vector>

#include "../paper_2609_34935_amd/csrc/qram_records.h"

using namespace qr;

static int failures = 0;
#define CHECK(cond)                                                   \
  do {                                                                \
    if (!(cond)) {                                                    \
      std::printf("FAIL %s:%d: %s\n", __FILE__, __LINE__, #cond);     \
      ++failures;                                                     \
    }                                                                 \
  } while (0)

namespace {

constexpr uint16_t GUARD = 0xBEEF;
constexpr int PAD = 64;  // guard words on each side of an address's records

struct Addr {
  int k, lmax, rec, K2;
  std::vector<uint16_t> buf;  // PAD guard | K2 records | PAD guard
  Addr(int k_, int lmax_) : k(k_), lmax(lmax_), K2(1 << k_) {
    rec = (lmax + 2 + k + 1 + 1) & ~1;  // the library's qubit record length
    buf.assign((size_t)2 * PAD + (size_t)K2 * rec, GUARD);
    for (int b = 0; b < K2; ++b) {
      uint16_t *r = rec_of(b);
      for (int j = 0; j < rec; ++j) r[j] = 0;
      for (int t = 0; t < k; ++t) r[2 + lmax + t] = (uint16_t)REC_EMPTY;
    }
  }
  uint16_t *rec_of(int b) { return buf.data() + PAD + (size_t)b * rec; }
  bool guards_intact() const {
    for (int j = 0; j < PAD; ++j)
      if (buf[j] != GUARD || buf[buf.size() - 1 - j] != GUARD) return false;
    return true;
  }
};

void test_rec_count() {
  uint32_t err = 0;
  CHECK(rec_count(5, 5, &err) == 5 && err == 0);
  CHECK(rec_count(0, 5, &err) == 0 && err == 0);
  CHECK(rec_count(6, 5, &err) == 5 && (err & ERR_LIST));
}

void test_class_mask() {
  // members (bus words) 0, 1, 2, 5 with split set D = 0b101: classes b & D
  const uint64_t members = (1u << 0) | (1u << 1) | (1u << 2) | (1u << 5);
  CHECK(class_mask(members, 5u) == ((1u << 0) | (1u << 1) | (1u << 5)));
  CHECK(class_mask(0, 5u) == 0);
}

// One class (D = 0) with address entries {3, 7} and tagged tokens 0 (site
// 9) and 1 (on the bus); split on token 0.
void test_class_split_valid() {
  Addr A(2, 6);
  uint16_t *r0 = A.rec_of(0);
  r0[0] = 2;
  r0[2] = 3;
  r0[3] = 7;
  r0[1] = (uint16_t)((0x2u) | (0x3u << 8));  // bus mask: token 1; tagged tokens 0, 1
  r0[2 + A.lmax + 0] = 9;
  r0[2 + A.lmax + 1] = (uint16_t)REC_EMPTY;
  uint32_t err = 0;
  rec_class_split(r0, A.rec, A.k, A.lmax, /*cl=*/1u, /*D=*/0u, /*X=*/1u, &err);
  CHECK(err == 0);
  CHECK(A.guards_intact());
  // class 0: token 0 dropped, list unchanged
  CHECK(r0[0] == 2 && r0[2] == 3 && r0[3] == 7);
  CHECK(r0[2 + A.lmax + 0] == REC_EMPTY);
  CHECK(((r0[1] >> 8) & 0xFFu) == 0x2u && (r0[1] & 0xFFu) == 0x2u);
  CHECK(r0[2 + A.lmax + A.k] == 1u);
  // class 1: token 0 kept as an ordinary entry
  const uint16_t *r1 = A.rec_of(1);
  CHECK(r1[0] == 3 && r1[2] == 3 && r1[3] == 7 && r1[4] == 9);
  CHECK(((r1[1] >> 8) & 0xFFu) == 0x2u && (r1[1] & 0xFFu) == 0x2u);
  CHECK(r1[2 + A.lmax + 0] == REC_EMPTY);
  CHECK(r1[2 + A.lmax + A.k] == 1u);
}

// Members 0..3 of class 0 become one list per bus word, each with the
// tagged tokens it carries that are in the tree.
void test_split_class_valid() {
  Addr A(2, 6);
  uint16_t *r0 = A.rec_of(0);
  r0[0] = 1;
  r0[2] = 4;
  r0[1] = (uint16_t)(0x0u | (0x3u << 8));  // tokens 0, 1 tagged, both in the tree
  r0[2 + A.lmax + 0] = 11;
  r0[2 + A.lmax + 1] = 13;
  std::vector<uint32_t> st(4 * 8, 0);
  uint32_t err = 0;
  rec_split_class(r0, A.rec, A.k, A.lmax, 0u, 0xFull, st.data(), 0u, 8u, &err);
  CHECK(err == 0);
  CHECK(A.guards_intact());
  for (int b = 0; b < 4; ++b) {
    const uint16_t *rb = A.rec_of(b);
    const int want = 1 + __builtin_popcount((unsigned)b);
    CHECK(rb[0] == want);
    CHECK(rb[2] == 4);
    int j = 3;
    if (b & 1) CHECK(rb[j++] == 11);
    if (b & 2) CHECK(rb[j++] == 13);
    CHECK(st[(size_t)b * 8] & W_SPLIT);
  }
}

// A damaged count (far above lmax) in the class being split.
void test_class_split_damaged() {
  for (uint16_t bad : {(uint16_t)7, (uint16_t)40, (uint16_t)0xFFFF}) {
    Addr A(2, 6);
    uint16_t *r0 = A.rec_of(0);
    r0[0] = bad;
    r0[1] = (uint16_t)(0x3u << 8);
    r0[2 + A.lmax + 0] = 9;
    r0[2 + A.lmax + 1] = 12;
    uint32_t err = 0;
    rec_class_split(r0, A.rec, A.k, A.lmax, 1u, 0u, 3u, &err);
    CHECK(err & ERR_LIST);
    CHECK(A.guards_intact());
    for (int b = 0; b < A.K2; ++b) CHECK(A.rec_of(b)[0] <= A.lmax);
  }
}

void test_split_class_damaged() {
  for (uint16_t bad : {(uint16_t)7, (uint16_t)40, (uint16_t)0xFFFF}) {
    Addr A(3, 8);
    uint16_t *r0 = A.rec_of(0);
    r0[0] = bad;
    r0[1] = (uint16_t)(0x7u << 8);
    for (int t = 0; t < 3; ++t) r0[2 + A.lmax + t] = (uint16_t)(20 + t);
    std::vector<uint32_t> st(8 * 4, 0);
    uint32_t err = 0;
    rec_split_class(r0, A.rec, A.k, A.lmax, 0u, 0xFFull, st.data(), 0u, 4u, &err);
    CHECK(err & ERR_LIST);
    CHECK(A.guards_intact());
    for (int b = 0; b < A.K2; ++b) CHECK(A.rec_of(b)[0] <= A.lmax);
  }
}

// A full list plus carried tokens beyond lmax: the extra entries are refused
// with ERR_LIST and nothing lands past the list.
void test_split_class_overflow() {
  Addr A(2, 4);
  uint16_t *r0 = A.rec_of(0);
  r0[0] = 4;
  for (int j = 0; j < 4; ++j) r0[2 + j] = (uint16_t)(30 + j);
  r0[1] = (uint16_t)(0x3u << 8);
  r0[2 + A.lmax + 0] = 40;
  r0[2 + A.lmax + 1] = 41;
  std::vector<uint32_t> st(4, 0);
  uint32_t err = 0;
  rec_split_class(r0, A.rec, A.k, A.lmax, 0u, 0xFull, st.data(), 0u, 1u, &err);
  CHECK(err & ERR_LIST);
  CHECK(A.guards_intact());
  for (int b = 0; b < 4; ++b) {
    CHECK(A.rec_of(b)[0] == 4);
    // the token slots after the list are untouched by the copy
    CHECK(A.rec_of(b)[2 + A.lmax + 0] == (b == 0 ? 40 : REC_EMPTY));
  }
}

}  // namespace

int main() {
  test_rec_count();
  test_class_mask();
  test_class_split_valid();
  test_split_class_valid();
  test_class_split_damaged();
  test_split_class_damaged();
  test_split_class_overflow();
  if (failures) {
    std::printf("%d checks failed\n", failures);
    return 1;
  }
  std::printf("ok\n");
  return 0;
}
