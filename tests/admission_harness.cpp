// Drives the serving loop's arena allocator and admission rule from stdin, for
// tests/test_admission_cpu.py.  Commands, one per line:
//   reset CAP | alloc BYTES | release OFF BYTES | stat | prefix ROOM MAX N F1 .. FN
#include <iostream>
#include <sstream>
#include <string>
#include <vector>

#include "admission.h"

int main()
{
    mmgap::serve::Arena a;
    std::string line;
    while (std::getline(std::cin, line)) {
        std::istringstream in(line);
        std::string op;
        in >> op;
        if (op == "reset") {
            size_t cap;
            in >> cap;
            a.reset(cap);
            std::cout << "ok\n";
        } else if (op == "alloc") {
            size_t b, off = 0;
            in >> b;
            if (a.alloc(b, &off)) std::cout << "ok " << off << "\n";
            else std::cout << "fail\n";
        } else if (op == "release") {
            size_t off, b;
            in >> off >> b;
            a.release(off, b);
            std::cout << "ok\n";
        } else if (op == "stat") {
            std::cout << a.free_bytes() << " " << a.largest_free() << " " << a.ranges() << "\n";
        } else if (op == "prefix") {
            size_t room;
            int mx, n;
            in >> room >> mx >> n;
            std::vector<size_t> f(n);
            for (auto &v : f) in >> v;
            std::cout << mmgap::serve::admit_prefix(f, room, mx) << "\n";
        }
    }
    return 0;
}
