// Drives the serving form's admission policy (serve_policy.h) from commands
// on stdin, one per line, for tests/test_serve_policy.py; prints one line
// per command.
//   new BUDGET MAX_INFLIGHT MAX_QUEUE
//   offer WS OUT            -> accept | too_large | queue_full
//   push TICKET WS OUT KEY SOLO
//   admit MAX_BATCH         -> batch T1 T2 ...   (admitted tickets, in order)
//   complete WS
//   release OUT
//   stats                   -> stats USED INFLIGHT QUEUED
#include "serve_policy.h"

#include <cstdio>
#include <iostream>
#include <memory>
#include <sstream>
#include <string>

int main() {
  std::unique_ptr<rlu_serve::Policy> pol;
  std::string line;
  while (std::getline(std::cin, line)) {
    std::istringstream in(line);
    std::string cmd;
    in >> cmd;
    if (cmd == "new") {
      size_t budget; int mi, mq;
      in >> budget >> mi >> mq;
      pol.reset(new rlu_serve::Policy(budget, mi, mq));
      std::printf("ok\n");
    } else if (cmd == "offer") {
      size_t ws, out;
      in >> ws >> out;
      const rlu_serve::Verdict v = pol->offer(ws, out);
      std::printf("%s\n", v == rlu_serve::Verdict::Accept ? "accept"
                          : v == rlu_serve::Verdict::TooLarge ? "too_large" : "queue_full");
    } else if (cmd == "push") {
      rlu_serve::Entry e;
      int solo;
      in >> e.ticket >> e.ws >> e.out >> e.key >> solo;
      e.solo = solo != 0;
      pol->push(e);
      std::printf("ok\n");
    } else if (cmd == "admit") {
      int mb;
      in >> mb;
      std::printf("batch");
      for (const rlu_serve::Entry& e : pol->admit(mb)) std::printf(" %llu", (unsigned long long)e.ticket);
      std::printf("\n");
    } else if (cmd == "complete") {
      size_t ws;
      in >> ws;
      pol->complete(ws);
      std::printf("ok\n");
    } else if (cmd == "release") {
      size_t out;
      in >> out;
      pol->release(out);
      std::printf("ok\n");
    } else if (cmd == "stats") {
      std::printf("stats %zu %d %zu\n", pol->used(), pol->inflight(), pol->queued());
    } else {
      std::printf("error %s\n", cmd.c_str());
    }
    std::fflush(stdout);
  }
  return 0;
}
